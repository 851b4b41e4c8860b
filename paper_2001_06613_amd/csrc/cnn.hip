// Learned temporal predictor: a convolutional encoder-decoder trained and
// run with hand-written bfloat16 MFMA kernels (float32 accumulation).
//
// Network (2-D): input [frame_l, frame_t, frame_r, u_l / h, u_r / h]
// (7 channels, NHWC, padded to 32), encoder convolutions 32/64/128/128
// (3x3, ReLU) with 2x2 average pooling, decoder with nearest 2x upsampling
// and skip concatenation [skip, up] (128/64/32), 1x1 head to the 2-channel
// correction in level pixels.  Parameters: one float32 vector, layer by
// layer W[tap][c_out][c_in] then b[c_out] (the order of the CPU reference).
//
// Convolution as an implicit GEMM on v_mfma_f32_32x32x16_bf16 (A = weights,
// B = input, D = output channels x pixels): a block computes 256 or 512
// consecutive output pixels (batch-flattened NHWC) by 32 or 64 output
// channels.  Per 16-channel chunk of the input it stages in LDS the input
// rows the taps reach (the pixel range widened by one image row and one
// pixel on each side) and the weights of every tap; each wave then runs the
// taps as MFMA steps with its operands reused across a 2 x 2 (or 4 x 1)
// grid of 32 x 32 output tiles.  The decoder's upsampled channels are read
// straight from the low-resolution tensor (nearest upsampling), so the
// concatenation [skip, up] is never materialised.  Backward data: the same
// kernel with the flipped, transposed weights.  Weight gradient: pixels
// are the reduction dimension; 32-pixel chunks of the upstream gradient and
// of the shifted input are staged in LDS transposed, split-K partials are
// summed in a fixed order by the Adam kernel.  Activations are bfloat16;
// gradients float32 (rounded to bfloat16 where they enter a matrix
// instruction).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <random>
#include <type_traits>
#include <vector>

#include "../../include/stml.h"
#include "launch.h"

namespace stml {
namespace cnn {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

constexpr int kCinPad = 32;
constexpr int kOutLd = 32;     // channels of the head output (D real)
constexpr int kMaxConvW = kMaxNetWidth;   // widest row a 3x3 conv stages

struct LayerDef {
  const char* name;
  int ci, co, k;
};
constexpr int kLayers = 15;
// 2-D table; in 3-D the first layer reads 3 + 2 x 3 channels and the head
// writes 3.
constexpr LayerDef kDefs[kLayers] = {
    {"e1a", 7, 32, 3},    {"e1b", 32, 32, 3},   {"e2a", 32, 64, 3},
    {"e2b", 64, 64, 3},   {"e3a", 64, 128, 3},  {"e3b", 128, 128, 3},
    {"e4a", 128, 128, 3}, {"e4b", 128, 128, 3}, {"d3a", 256, 128, 3},
    {"d3b", 128, 128, 3}, {"d2a", 192, 64, 3},  {"d2b", 64, 64, 3},
    {"d1a", 96, 32, 3},   {"d1b", 32, 32, 3},   {"head", 32, 2, 1},
};
enum { E1A, E1B, E2A, E2B, E3A, E3B, E4A, E4B, D3A, D3B, D2A, D2B, D1A, D1B,
       HEAD };

static LayerDef layer_def(int dim, int i) {
  LayerDef d = kDefs[i];
  if (i == E1A) d.ci = 3 + 2 * dim;
  if (i == HEAD) d.co = dim;
  return d;
}
// taps of a layer with kernel size k
static int layer_taps(int dim, int k) { return dim == 3 ? k * k * k : k * k; }

static int rup(int v, int m) { return (v + m - 1) / m * m; }

// ------------------------------------------------------------ kernels

__device__ __forceinline__ bf16x8 load8(const bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}
__device__ __forceinline__ bf16x8 load8(const float* p) {
  f32x4 a = *reinterpret_cast<const f32x4*>(p);
  f32x4 b = *reinterpret_cast<const f32x4*>(p + 4);
  bf16x8 r;
  r[0] = (bf16)a[0]; r[1] = (bf16)a[1]; r[2] = (bf16)a[2]; r[3] = (bf16)a[3];
  r[4] = (bf16)b[0]; r[5] = (bf16)b[1]; r[6] = (bf16)b[2]; r[7] = (bf16)b[3];
  return r;
}

// Input channels of a convolution: [0, split) from a0 at the layer's
// resolution, [split, cin_p) from a1 at half resolution (pixel (y, x) reads
// a1's (y / 2, x / 2): nearest upsampling).  split is a multiple of 16.
template <class TX>
struct ConvSrc {
  const TX* a0;
  int ld0, off0;
  const TX* a1;
  int ld1, off1;
  int split;
};

constexpr int kRowLd = 24;      // LDS row: 16 channels + 8 of padding

// Y[p][yoff + co] = act(bias[co] + sum_tap sum_ci X[p + off(tap)][ci]
//                   Wt[tap][co][ci]) with zero padding, p = (b, z, y, x)
// flattened (z absent in 2-D: Z = 1, KZ = 1).  3-D taps (KZ = 3) are run as
// three planes of K x K taps: for plane dz the staged rows are those of the
// 2-D case shifted by dz H W, so the LDS footprint does not grow.  Block:
// 128 PS pixels x 32 CS output channels; wave w owns pixel subtiles
// PS w .. PS w + PS - 1 (32 pixels each) and all CS channel subtiles.
// Requires W <= 256 (LDS rows of the halo), cin_p % 16 == 0.
template <int K, int KZ, int CS, int PS, class TX, bool OUT_F32, bool RELU>
__global__ __launch_bounds__(256) void conv_kernel(
    ConvSrc<TX> src, int cin_p, const bf16* __restrict__ Wt,
    const float* __restrict__ bias, int cout, int cout_p,
    void* __restrict__ Yv, int yld, int yoff, int B, int Z, int H, int W) {
  constexpr int TP = 128 * PS;           // pixels per block
  constexpr int COB = 32 * CS;           // output channels per block
  constexpr int K2 = K * K;
  extern __shared__ __align__(16) bf16 lds[];
  const int R = K == 3 ? W + 1 : 0;      // halo of the flattened range
  const int NR = TP + 2 * R;             // staged rows
  bf16* act = lds;
  bf16* wl = lds + (size_t)NR * kRowLd;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ln = lane & 31, kh = lane >> 5;
  const long long HW = (long long)H * W;
  const long long ZHW = (long long)Z * HW;
  const long long P = (long long)B * ZHW;
  const long long p0 = (long long)blockIdx.x * TP;
  const int co_base = blockIdx.y * COB;
  // this lane's pixels
  int pz[PS], py[PS], pxx[PS];
  bool pv[PS];
#pragma unroll
  for (int s = 0; s < PS; ++s) {
    long long p = p0 + 32 * (PS * w + s) + ln;
    pv[s] = p < P;
    long long rem = pv[s] ? p % ZHW : 0;
    pz[s] = (int)(rem / HW);
    rem -= (long long)pz[s] * HW;
    py[s] = (int)(rem / W);
    pxx[s] = (int)(rem - (long long)py[s] * W);
  }
  f32x16 acc[PS][CS];
#pragma unroll
  for (int s = 0; s < PS; ++s)
#pragma unroll
    for (int c = 0; c < CS; ++c)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[s][c][i] = 0.f;
  const bf16x8 zero = {};
  const int H1 = H >> 1, W1 = W >> 1, Z1 = KZ == 3 ? Z >> 1 : 1;
  for (int c0 = 0; c0 < cin_p; c0 += 16) {
    const bool hi = c0 >= src.split;
    const TX* sp = hi ? src.a1 : src.a0;
    const int sld = hi ? src.ld1 : src.ld0;
    const int soff = hi ? src.off1 + c0 - src.split : src.off0 + c0;
    for (int pl = 0; pl < KZ; ++pl) {
      const int dz = pl - KZ / 2;
      // stage the input rows [p0 - R, p0 + TP + R) + dz H W of this chunk
      const long long qb = p0 - R + dz * HW;
      for (int e = tid; e < 2 * NR; e += 256) {
        const int row = e >> 1, hf = e & 1;
        const long long q = qb + row;
        bf16x8 v = zero;
        if (q >= 0 && q < P) {
          long long idx = q;
          if (hi) {
            const long long b = q / ZHW;
            long long rem = q - b * ZHW;
            const int zz = (int)(rem / HW);
            rem -= (long long)zz * HW;
            const int yy = (int)(rem / W), xx = (int)(rem - (long long)yy * W);
            idx = ((b * Z1 + (KZ == 3 ? zz >> 1 : 0)) * H1 + (yy >> 1)) * W1 +
                  (xx >> 1);
          }
          v = load8(sp + idx * sld + soff + 8 * hf);
        }
        *reinterpret_cast<bf16x8*>(act + row * kRowLd + 8 * hf) = v;
      }
      // stage the weights of the plane's taps for the block's channels
      for (int e = tid; e < 2 * K2 * COB; e += 256) {
        const int row = e >> 1, hf = e & 1;
        const int tap = row / COB, co = row - tap * COB;
        *reinterpret_cast<bf16x8*>(wl + row * kRowLd + 8 * hf) =
            load8(Wt + ((size_t)(pl * K2 + tap) * cout_p + co_base + co) *
                           cin_p +
                  c0 + 8 * hf);
      }
      __syncthreads();
      bool zok[PS];
#pragma unroll
      for (int s = 0; s < PS; ++s) {
        const int zz = pz[s] + dz;
        zok[s] = pv[s] && zz >= 0 && zz < Z;
      }
#pragma unroll
      for (int tap = 0; tap < K2; ++tap) {
        const int dy = tap / K - K / 2, dx = tap % K - K / 2;
        bf16x8 bop[PS];
#pragma unroll
        for (int s = 0; s < PS; ++s) {
          const int yy = py[s] + dy, xx = pxx[s] + dx;
          const bool ok = zok[s] && yy >= 0 && yy < H && xx >= 0 && xx < W;
          const int row = 32 * (PS * w + s) + ln + R + dy * W + dx;
          bop[s] = ok ? *reinterpret_cast<const bf16x8*>(act + row * kRowLd +
                                                         8 * kh)
                      : zero;
        }
#pragma unroll
        for (int c = 0; c < CS; ++c) {
          const bf16x8 aop = *reinterpret_cast<const bf16x8*>(
              wl + (tap * COB + 32 * c + ln) * kRowLd + 8 * kh);
#pragma unroll
          for (int s = 0; s < PS; ++s)
            acc[s][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                aop, bop[s], acc[s][c], 0, 0, 0);
        }
      }
      __syncthreads();
    }
  }
  // D[co][pixel]: lane holds pixel ln, channels 8 g + 4 kh + (0..3)
#pragma unroll
  for (int s = 0; s < PS; ++s) {
    if (!pv[s]) continue;
    const long long p = p0 + 32 * (PS * w + s) + ln;
    const size_t obase = (size_t)p * yld + yoff;
#pragma unroll
    for (int c = 0; c < CS; ++c)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int co = co_base + 32 * c + 8 * g + 4 * kh;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float bb = (bias && co + i < cout) ? bias[co + i] : 0.f;
          v[i] = acc[s][c][4 * g + i] + bb;
          if (RELU) v[i] = v[i] > 0.f ? v[i] : 0.f;
        }
        if (OUT_F32) {
          *reinterpret_cast<f32x4*>(reinterpret_cast<float*>(Yv) + obase +
                                    co) = f32x4{v[0], v[1], v[2], v[3]};
        } else {
          *reinterpret_cast<bf16x4*>(reinterpret_cast<bf16*>(Yv) + obase +
                                     co) =
              bf16x4{(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
        }
      }
  }
}

constexpr int kWChunk = 128;    // pixels staged per step of the weight gradient
constexpr int kWLd = kWChunk + 8;

// part[s][tap][co][ci] = sum over the pixels of split s of
//   bf16(dP[p][poff + co]) * X[p + off(tap)][ci]   (zero padding; KZ K K
//   taps, KZ = 3 for volumes)
// Block: 64 output channels x 64 input channels of one tap; wave w owns
// output channels 16w..16w+15 and all four 16-channel input subtiles.  Per
// step 128 pixels of dP and of the shifted input are staged transposed
// (channel-major) in LDS: thread t loads 32 contiguous channels of pixel
// t % 128.
template <int K, int KZ>
__global__ __launch_bounds__(256) void wgrad_kernel(
    const float* __restrict__ dP, int pld, int poff, int cout_p,
    ConvSrc<bf16> X, int cin_p, int B, int Z, int H, int W,
    int chunks_per_split, float* __restrict__ part) {
  __shared__ __align__(16) bf16 As[64][kWLd];
  __shared__ __align__(16) bf16 Bs[64][kWLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nco = (cout_p + 63) / 64, nci = (cin_p + 63) / 64;
  int t = blockIdx.y;
  const int cib = t % nci;
  t /= nci;
  const int cob = t % nco;
  const int tap = t / nco;
  const int dz = tap / (K * K) - KZ / 2;
  const int dy = (tap / K) % K - K / 2, dx = tap % K - K / 2;
  const int s = blockIdx.x;
  const long long HW = (long long)H * W, ZHW = Z * HW;
  const long long P = (long long)B * ZHW;
  const long long nchunks = (P + kWChunk - 1) / kWChunk;
  const long long c_beg = (long long)s * chunks_per_split;
  long long c_end = c_beg + chunks_per_split;
  if (c_end > nchunks) c_end = nchunks;
  const int kq = (lane >> 4) * 8;
  f32x4 acc[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int sp = threadIdx.x & (kWChunk - 1), c32 = (threadIdx.x >> 7) * 32;
  const int co0 = cob * 64 + c32, ci0 = cib * 64 + c32;
  for (long long ch = c_beg; ch < c_end; ++ch) {
    const long long p = ch * kWChunk + sp;
    {
      float v[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) v[i] = 0.f;
      if (p < P && co0 < cout_p) {
        const float* src = dP + p * pld + poff + co0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          f32x4 a = *reinterpret_cast<const f32x4*>(src + 4 * q);
          v[4 * q] = a[0];
          v[4 * q + 1] = a[1];
          v[4 * q + 2] = a[2];
          v[4 * q + 3] = a[3];
        }
      }
#pragma unroll
      for (int i = 0; i < 32; ++i) As[c32 + i][sp] = (bf16)v[i];
    }
    {
      bf16x8 v[4] = {};
      if (p < P && ci0 < cin_p) {
        const long long pb = p / ZHW;
        long long rem = p - pb * ZHW;
        const int zz = (int)(rem / HW) + dz;
        rem %= HW;
        const int yy = (int)(rem / W) + dy, xx = (int)(rem % W) + dx;
        if (zz >= 0 && zz < Z && yy >= 0 && yy < H && xx >= 0 && xx < W) {
          const int Z1 = KZ == 3 ? Z >> 1 : 1, z1 = KZ == 3 ? zz >> 1 : 0;
          const bf16* src =
              ci0 < X.split
                  ? X.a0 + ((((size_t)pb * Z + zz) * H + yy) * W + xx) *
                               X.ld0 + X.off0 + ci0
                  : X.a1 +
                        ((((size_t)pb * Z1 + z1) * (H >> 1) + (yy >> 1)) *
                             (W >> 1) + (xx >> 1)) * X.ld1 + X.off1 + ci0 -
                        X.split;
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = load8(src + 8 * q);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) Bs[c32 + 8 * q + i][sp] = v[q][i];
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < kWChunk; k0 += 32) {
      const bf16x8 aop = *reinterpret_cast<const bf16x8*>(
          &As[16 * w + (lane & 15)][k0 + kq]);
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const bf16x8 bop = *reinterpret_cast<const bf16x8*>(
            &Bs[16 * n + (lane & 15)][k0 + kq]);
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, acc[n], 0,
                                                         0, 0);
      }
    }
    __syncthreads();
  }
  const int K2 = KZ * K * K;
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const int ci = cib * 64 + 16 * n + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = cob * 64 + 16 * w + (lane >> 4) * 4 + i;
      if (co < cout_p && ci < cin_p)
        part[(((size_t)s * K2 + tap) * cout_p + co) * cin_p + ci] = acc[n][i];
    }
  }
}

// bpart[s][co] = sum over the pixels of split s of bf16(dP[p][poff + co])
__global__ void bias_grad_kernel(const float* __restrict__ dP, int pld,
                                 int poff, int cout_p, long long P,
                                 long long pix_per_split,
                                 float* __restrict__ bpart) {
  const int co = threadIdx.x;
  if (co >= cout_p) return;
  const long long p0 = (long long)blockIdx.x * pix_per_split;
  long long p1 = p0 + pix_per_split;
  if (p1 > P) p1 = P;
  float acc = 0.f;
#pragma unroll 8
  for (long long p = p0; p < p1; ++p)
    acc += (float)(bf16)dP[p * pld + poff + co];
  bpart[(size_t)blockIdx.x * cout_p + co] = acc;
}

// gb[co] = sum_s bpart[s][co]: one wave per channel, lane i sums the
// splits i, i + 64, ..., then a fixed butterfly (deterministic order).
__global__ __launch_bounds__(64) void bias_reduce_kernel(
    const float* __restrict__ bpart, int bsplit, int cout_p,
    float* __restrict__ gb) {
  const int co = blockIdx.x, lane = threadIdx.x;
  float acc = 0.f;
  for (int s = lane; s < bsplit; s += 64) acc += bpart[(size_t)s * cout_p + co];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) gb[co] = acc;
}

struct AdamArgs {
  float lr, b1, b2, eps, c1, c2;   // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
  int apply;
};

// Gradient of one layer from the split partials (fixed summation order) and
// the reduced bias gradient gb,
// optional copy out, Adam step on the float32 master, and the bfloat16
// forward (Wt[tap][co_p][ci_p]) and backward (Wb[K2-1-tap][ci_p][co_p])
// weight copies.
__global__ void adam_layer_kernel(const float* __restrict__ part, int nsplit,
                                  const float* __restrict__ gb, int K2, int cout, int cin, int cout_p,
                                  int cin_p, float* __restrict__ master,
                                  float* __restrict__ m, float* __restrict__ v,
                                  float* __restrict__ grad_out, bf16* Wt,
                                  bf16* Wb, AdamArgs a) {
  const int nw = K2 * cout * cin;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nw + cout) return;
  float g = 0.f;
  int tap = 0, co, ci = 0;
  if (e < nw) {
    tap = e / (cout * cin);
    int r = e - tap * cout * cin;
    co = r / cin;
    ci = r - co * cin;
    const size_t stride = (size_t)K2 * cout_p * cin_p;
    const float* pp = part + ((size_t)tap * cout_p + co) * cin_p + ci;
#pragma unroll 8
    for (int s = 0; s < nsplit; ++s) g += pp[(size_t)s * stride];
  } else {
    co = e - nw;
    g = gb[co];
  }
  if (grad_out) grad_out[e] = g;
  if (!a.apply) return;
  float mm = a.b1 * m[e] + (1.f - a.b1) * g;
  float vv = a.b2 * v[e] + (1.f - a.b2) * g * g;
  m[e] = mm;
  v[e] = vv;
  float wv = master[e] - a.lr * (mm * a.c1) / (sqrtf(vv * a.c2) + a.eps);
  master[e] = wv;
  if (e < nw) {
    Wt[((size_t)tap * cout_p + co) * cin_p + ci] = (bf16)wv;
    Wb[((size_t)(K2 - 1 - tap) * cin_p + ci) * cout_p + co] = (bf16)wv;
  }
}

// Bfloat16 weight copies of one layer from the float32 master.
__global__ void weights_from_master_kernel(const float* __restrict__ master,
                                           int K2, int cout, int cin,
                                           int cout_p, int cin_p, bf16* Wt,
                                           bf16* Wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K2 * cout * cin) return;
  int tap = e / (cout * cin);
  int r = e - tap * cout * cin;
  int co = r / cin, ci = r - co * cin;
  bf16 wv = (bf16)master[e];
  Wt[((size_t)tap * cout_p + co) * cin_p + ci] = wv;
  Wb[((size_t)(K2 - 1 - tap) * cin_p + ci) * cout_p + co] = wv;
}

__global__ void zero_f32_kernel(float* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t st = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = 0.f;
}

// dP[p][off + c] *= (post[p][poff + c] > 0), c < C
__global__ void relu_bwd_kernel(float* __restrict__ dP, int ld, int off,
                                const bf16* __restrict__ post, int pld,
                                int poff, int C, long long P) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < P * C; i += st) {
    long long p = i / C;
    int c = (int)(i - p * C);
    if (!((float)post[p * pld + poff + c] > 0.f)) dP[p * ld + off + c] = 0.f;
  }
}

// 2x2 (2-D, Z = 1, DZ = 1) or 2x2x2 (3-D, DZ = 2) average pooling,
// bfloat16 in and out; the block sum is formed in float32 (exact for four
// bfloat16 values, and for eight of like magnitude).
template <int DZ>
__global__ void pool_kernel(const bf16* __restrict__ X, int xld, int xoff,
                            int C, int B, int Z, int H, int W,
                            bf16* __restrict__ Y, int yld) {
  const int Zo = Z / DZ, Ho = H / 2, Wo = W / 2;
  long long n = (long long)B * Zo * Ho * Wo * C;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    int c = (int)(i % C);
    long long q = i / C;
    int xo = (int)(q % Wo);
    long long r = q / Wo;
    int yo = (int)(r % Ho);
    r /= Ho;
    int zo = (int)(r % Zo);
    int b = (int)(r / Zo);
    float sum = 0.f;
#pragma unroll
    for (int k = 0; k < DZ; ++k) {
      size_t p00 = ((((size_t)b * Z + DZ * zo + k) * H + 2 * yo) * W + 2 * xo);
      sum += (float)X[p00 * xld + xoff + c] +
             (float)X[(p00 + 1) * xld + xoff + c] +
             (float)X[(p00 + W) * xld + xoff + c] +
             (float)X[(p00 + W + 1) * xld + xoff + c];
    }
    Y[q * yld + c] = (bf16)(sum * (DZ == 2 ? 0.125f : 0.25f));
  }
}

// dX[DZ z + k][2y+i][2x+j][off + c] += dY[z][y][x][c] / 2^d
template <int DZ>
__global__ void pool_bwd_add_kernel(const float* __restrict__ dY, int C,
                                    int B, int Z, int H, int W,
                                    float* __restrict__ dX, int dld,
                                    int doff) {
  long long n = (long long)B * Z * H * W * C;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  const int Zi = Z / DZ, Hi = H / 2, Wi = W / 2;
  for (; i < n; i += st) {
    int c = (int)(i % C);
    long long q = i / C;
    int x = (int)(q % W);
    long long r = q / W;
    int y = (int)(r % H);
    r /= H;
    int z = (int)(r % Z);
    int b = (int)(r / Z);
    float g = dY[((((size_t)b * Zi + z / DZ) * Hi + y / 2) * Wi + x / 2) * C +
                 c] *
              (DZ == 2 ? 0.125f : 0.25f);
    dX[q * dld + doff + c] += g;
  }
}

// dX[z][y][x][c] = sum of dY[DZ z + k][2y+i][2x+j][off + c]
template <int DZ>
__global__ void up_bwd_kernel(const float* __restrict__ dY, int dld, int doff,
                              int C, int B, int Z, int H, int W,
                              float* __restrict__ dX) {
  const int Zo = Z / DZ, Ho = H / 2, Wo = W / 2;
  long long n = (long long)B * Zo * Ho * Wo * C;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    int c = (int)(i % C);
    long long q = i / C;
    int xo = (int)(q % Wo);
    long long r = q / Wo;
    int yo = (int)(r % Ho);
    r /= Ho;
    int zo = (int)(r % Zo);
    int b = (int)(r / Zo);
    float sum = 0.f;
#pragma unroll
    for (int k = 0; k < DZ; ++k) {
      size_t p00 = ((((size_t)b * Z + DZ * zo + k) * H + 2 * yo) * W + 2 * xo);
      sum += dY[p00 * dld + doff + c] + dY[(p00 + 1) * dld + doff + c] +
             dY[(p00 + W) * dld + doff + c] +
             dY[(p00 + W + 1) * dld + doff + c];
    }
    dX[q * C + c] = sum;
  }
}

// Mean squared error of the nc-channel head (ld kOutLd) against tgt
// [P][nc]; dout = 2 (out - tgt) / (nc P) in channels < nc and 0 elsewhere;
// per-block float64 partial of the squared error.
__global__ __launch_bounds__(256) void loss_kernel(
    const float* __restrict__ out, const float* __restrict__ tgt, long long P,
    int nc, float* __restrict__ dout, double* __restrict__ part) {
  const double inv = 1.0 / ((double)nc * (double)P);
  double acc = 0.0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < kOutLd; ++c) {
      float g = 0.f;
      if (c < nc) {
        double d = (double)out[p * kOutLd + c] - (double)tgt[p * nc + c];
        acc += d * d;
        g = (float)(2.0 * d * inv);
      }
      dout[p * kOutLd + c] = g;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv;
}

__global__ void loss_final_kernel(const double* __restrict__ part, int nb,
                                  double* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += part[i];
    *loss = s;
  }
}

// Network input from planar float32 channels [B][C][N] (C <= 32, N pixels
// or voxels per frame), channels last.
__global__ void pack_input_kernel(const float* __restrict__ x, int C, int B,
                                  long long N, bf16* __restrict__ xin) {
  long long n = (long long)B * N * kCinPad;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    int c = (int)(i % kCinPad);
    long long p = i / kCinPad;
    long long b = p / N;
    long long hw = p - b * N;
    float v = c < C ? x[(b * C + c) * N + hw] : 0.f;
    xin[i] = (bf16)v;
  }
}

// Inputs of frames t with registered neighbours l < t < r (D components,
// N voxels per frame): [T_l, T_t, T_r, u_l / h, u_r / h] (3 + 2D channels),
// the linear-interpolation base u_b = w_l u_l + w_r u_r ([B][D][N]) and, if
// U_t is wanted, the target correction (u_t - u_b) / h ([B][N][D]).
__global__ void assemble_kernel(const float* __restrict__ T,
                                const float* __restrict__ U,
                                const int* __restrict__ tlr, int B, int D,
                                long long N, double inv_h,
                                bf16* __restrict__ xin,
                                float* __restrict__ base,
                                float* __restrict__ tgt) {
  long long n = (long long)B * N;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    int b = (int)(i / N);
    long long hw = i - (long long)b * N;
    int t = tlr[3 * b], l = tlr[3 * b + 1], r = tlr[3 * b + 2];
    double wl = (double)(r - t) / (r - l), wr = (double)(t - l) / (r - l);
    bf16* o = xin + i * kCinPad;
    o[0] = (bf16)T[(size_t)l * N + hw];
    o[1] = (bf16)T[(size_t)t * N + hw];
    o[2] = (bf16)T[(size_t)r * N + hw];
    for (int a = 0; a < D; ++a) {
      double ul = U[((size_t)l * D + a) * N + hw];
      double ur = U[((size_t)r * D + a) * N + hw];
      o[3 + a] = (bf16)(float)(ul * inv_h);
      o[3 + D + a] = (bf16)(float)(ur * inv_h);
      double ub = wl * ul + wr * ur;
      base[((size_t)b * D + a) * N + hw] = (float)ub;
      if (tgt) {
        double ut = U[((size_t)t * D + a) * N + hw];
        tgt[i * D + a] = (float)((ut - ub) * inv_h);
      }
    }
    for (int c = 3 + 2 * D; c < kCinPad; ++c) o[c] = (bf16)0.f;
  }
}

// u_t = base + h * correction, written into the all-frame field Uout.
__global__ void emit_kernel(const float* __restrict__ base,
                            const float* __restrict__ out,
                            const int* __restrict__ tlr, int B, int D,
                            long long N, double h, float* __restrict__ Uout) {
  long long n = (long long)B * N;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    int b = (int)(i / N);
    long long hw = i - (long long)b * N;
    int t = tlr[3 * b];
    for (int a = 0; a < D; ++a)
      Uout[((size_t)t * D + a) * N + hw] =
          (float)((double)base[((size_t)b * D + a) * N + hw] +
                  h * (double)out[i * kOutLd + a]);
  }
}

static int gridsz(long long n) {
  long long nb = (n + 255) / 256;
  return (int)(nb < 1 ? 1 : (nb > 8192 ? 8192 : nb));
}

}  // namespace cnn
}  // namespace stml

// ================================================================ network

using namespace stml;
using namespace stml::cnn;

namespace {

struct Buf {
  bf16* a;   // activation (bfloat16)
  float* g;  // gradient (float32)
  int ld;
  int level;
};

struct Layer {
  int ci, co, k, taps, ci_p, co_p;
  size_t woff, boff;      // offsets into the flat parameter vector
  bf16 *Wt, *Wb;
};

}  // namespace

// Frames are Z x H x W (Z = 1 for images), channels last.
struct stml_net {
  int dim = 2, maxB = 0, maxZ = 1, maxH = 0, maxW = 0;
  hipStream_t stream = nullptr;
  size_t nparam = 0;
  float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  Layer L[kLayers];
  // activations and gradients
  Buf xin, e1a, c1, p1, e2a, c2, p2, e3a, c3, p3, e4a, e4b, d3a, d3b, d2a,
      d2b, d1a, d1b;
  float* out = nullptr;     // head output [P][kOutLd]
  float* dout = nullptr;
  float* base = nullptr;    // [B][D][N]
  float* tgt = nullptr;     // [B][N][D]
  int* tlr = nullptr;       // device triples
  int* htlr = nullptr;      // pinned host staging
  float* wpart = nullptr;
  size_t wpart_cap = 0;     // floats
  float* bpart = nullptr;
  size_t bpart_cap = 0;
  float* gb = nullptr;      // reduced bias gradient of one layer
  double* lpart = nullptr;
  double* dloss = nullptr;
  double* hloss = nullptr;  // pinned
  int step = 0;
  int curB = 0, curZ = 1, curH = 0, curW = 0;
};

namespace {

constexpr size_t kAlignN = 256;
size_t alignn(size_t v) { return (v + kAlignN - 1) / kAlignN * kAlignN; }

struct NetLayout {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    size_t o = off;
    off = alignn(off + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

constexpr size_t kWpartCap = (size_t)6 << 20;   // floats of split partials
constexpr int kBSplit = 1024;

long long max_pixels(const stml_net* n) {
  return (long long)n->maxB * n->maxZ * n->maxH * n->maxW;
}

// Frames a batch may hold: every frame has at least 8^d pixels.
size_t max_frames(const stml_net* n) {
  return (size_t)(max_pixels(n) / (n->dim == 3 ? 512 : 64));
}

size_t net_layout(stml_net* n, char* base) {
  NetLayout lo;
  lo.base = base;
  size_t np = 0;
  for (int i = 0; i < kLayers; ++i) {
    const LayerDef d = layer_def(n->dim, i);
    Layer& l = n->L[i];
    l.ci = d.ci;
    l.co = d.co;
    l.k = d.k;
    l.taps = layer_taps(n->dim, d.k);
    l.ci_p = rup(d.ci, 32);
    l.co_p = rup(d.co, 32);
    l.woff = np;
    np += (size_t)l.taps * d.co * d.ci;
    l.boff = np;
    np += d.co;
  }
  n->nparam = np;
  n->master = lo.take<float>(np);
  n->m = lo.take<float>(np);
  n->v = lo.take<float>(np);
  n->grad = lo.take<float>(np);
  for (int i = 0; i < kLayers; ++i) {
    Layer& l = n->L[i];
    size_t nw = (size_t)l.taps * l.co_p * l.ci_p;
    l.Wt = lo.take<bf16>(nw);
    l.Wb = lo.take<bf16>(nw);
  }
  const size_t P0 = (size_t)max_pixels(n);
  auto buf = [&](Buf& b, int ch, int level) {
    size_t P = P0 >> (n->dim * level);
    b.a = lo.take<bf16>(P * ch);
    b.g = lo.take<float>(P * ch);
    b.ld = ch;
    b.level = level;
  };
  buf(n->xin, 32, 0);
  buf(n->e1a, 32, 0);
  buf(n->c1, 96, 0);
  buf(n->p1, 32, 1);
  buf(n->e2a, 64, 1);
  buf(n->c2, 192, 1);
  buf(n->p2, 64, 2);
  buf(n->e3a, 128, 2);
  buf(n->c3, 256, 2);
  buf(n->p3, 128, 3);
  buf(n->e4a, 128, 3);
  buf(n->e4b, 128, 3);
  buf(n->d3a, 128, 2);
  buf(n->d3b, 128, 2);
  buf(n->d2a, 64, 1);
  buf(n->d2b, 64, 1);
  buf(n->d1a, 32, 0);
  buf(n->d1b, 32, 0);
  n->out = lo.take<float>(P0 * kOutLd);
  n->dout = lo.take<float>(P0 * kOutLd);
  n->base = lo.take<float>(P0 * n->dim);
  n->tgt = lo.take<float>(P0 * n->dim);
  n->tlr = lo.take<int>(3 * max_frames(n));
  n->wpart_cap = kWpartCap;
  n->wpart = lo.take<float>(kWpartCap);
  n->bpart_cap = (size_t)kBSplit * 128;
  n->bpart = lo.take<float>(n->bpart_cap);
  n->gb = lo.take<float>(256);
  n->lpart = lo.take<double>(8192);
  n->dloss = lo.take<double>(1);
  return lo.off;
}

#define NET_OK(call)                     \
  do {                                   \
    if ((call) != hipSuccess) return STML_EDEVICE; \
  } while (0)

// Extents of resolution level lev (0 = full).
struct Ext {
  int z, h, w;
  long long pix() const { return (long long)z * h * w; }
};
Ext level_ext(const stml_net* n, int Z, int H, int W, int lev) {
  return Ext{n->dim == 3 ? Z >> lev : 1, H >> lev, W >> lev};
}

// One convolution: K x K (x K in 3-D) taps, input src (cin_p channels),
// weights Wmat[tap][cout_p][cin_p], output Y (yld, yoff) in float32 or
// bfloat16.  64-channel blocks (2 x 2 tiles per wave) when cout_p allows,
// else 32-channel blocks of 512 pixels (4 x 1 tiles per wave).
template <class TX>
hipError_t conv_launch(stml_net* n, int K, const ConvSrc<TX>& src, int cin_p,
                       const bf16* Wmat, const float* bias, int cout,
                       int cout_p, void* Y, bool y_f32, int yld, int yoff,
                       bool relu, int B, Ext e) {
  if ((K != 1 && K != 3) || cin_p % 16 || cout_p % 32 || src.split % 16 ||
      (K == 3 && e.w > kMaxConvW))
    return hipErrorInvalidValue;
  const bool vol = n->dim == 3 && K == 3;
  const bool wide = cout_p % 64 == 0;
  const int TP = wide ? 256 : 512, COB = wide ? 64 : 32;
  const int R = K == 3 ? e.w + 1 : 0;
  const size_t lds = ((size_t)(TP + 2 * R) + (size_t)K * K * COB) * kRowLd *
                     sizeof(bf16);
  const long long P = (long long)B * e.pix();
  dim3 grid((unsigned)((P + TP - 1) / TP), cout_p / COB);
  hipStream_t s = n->stream;
  constexpr bool F = std::is_same<TX, float>::value;
#define CONV_CASE(KK, KZ, CSS, PSS, OF, RL)                                  \
  conv_kernel<KK, KZ, CSS, PSS, TX, OF, RL><<<grid, 256, lds, s>>>(         \
      src, cin_p, Wmat, bias, cout, cout_p, Y, yld, yoff, B, e.z, e.h, e.w)
#define CONV_DIMS(CSS, PSS, OF, RL)          \
  do {                                       \
    if (vol) CONV_CASE(3, 3, CSS, PSS, OF, RL); \
    else CONV_CASE(3, 1, CSS, PSS, OF, RL);  \
  } while (0)
  if (!F && K == 3 && !y_f32 && relu) {
    if (wide) CONV_DIMS(2, 2, false, true);
    else CONV_DIMS(1, 4, false, true);
  } else if (K == 3 && y_f32 && !relu) {
    if (wide) CONV_DIMS(2, 2, true, false);
    else CONV_DIMS(1, 4, true, false);
  } else if (K == 1 && y_f32 && !relu && !wide) {
    CONV_CASE(1, 1, 1, 4, true, false);
  } else {
    return hipErrorInvalidValue;
  }
#undef CONV_DIMS
#undef CONV_CASE
  return hipGetLastError();
}

ConvSrc<bf16> one_src(const Buf& b, int off, int C) {
  return ConvSrc<bf16>{b.a, b.ld, off, nullptr, 0, 0, C};
}

// [skip channels of b, upsampled channels of low]
ConvSrc<bf16> cat_src(const Buf& b, int skipC, const Buf& low) {
  return ConvSrc<bf16>{b.a, b.ld, 0, low.a, low.ld, 0, skipC};
}

template <class... A>
hipError_t pool_launch(int dim, long long nthreads, hipStream_t s, A... a) {
  if (dim == 3)
    pool_kernel<2><<<gridsz(nthreads), 256, 0, s>>>(a...);
  else
    pool_kernel<1><<<gridsz(nthreads), 256, 0, s>>>(a...);
  return hipGetLastError();
}
template <class... A>
hipError_t pool_bwd_launch(int dim, long long nthreads, hipStream_t s,
                           A... a) {
  if (dim == 3)
    pool_bwd_add_kernel<2><<<gridsz(nthreads), 256, 0, s>>>(a...);
  else
    pool_bwd_add_kernel<1><<<gridsz(nthreads), 256, 0, s>>>(a...);
  return hipGetLastError();
}
template <class... A>
hipError_t up_bwd_launch(int dim, long long nthreads, hipStream_t s, A... a) {
  if (dim == 3)
    up_bwd_kernel<2><<<gridsz(nthreads), 256, 0, s>>>(a...);
  else
    up_bwd_kernel<1><<<gridsz(nthreads), 256, 0, s>>>(a...);
  return hipGetLastError();
}

// Forward through every layer for B frames of Z x H x W (multiples of 8).
int net_forward(stml_net* n, int B, int Z, int H, int W) {
  auto conv3 = [&](int li, const ConvSrc<bf16>& in, int lev, Buf& outb,
                   int ooff) {
    const Layer& l = n->L[li];
    return conv_launch(n, 3, in, l.ci_p, l.Wt, n->master + l.boff, l.co,
                       l.co_p, outb.a, false, outb.ld, ooff, true, B,
                       level_ext(n, Z, H, W, lev));
  };
  auto pool = [&](const Buf& in, int ioff, int C, Buf& outb) {
    const Ext e = level_ext(n, Z, H, W, in.level);
    return pool_launch(n->dim, ((long long)B * e.pix() >> n->dim) * C,
                       n->stream,
                       (const bf16*)in.a, in.ld, ioff, C, B, e.z, e.h,
                       e.w, outb.a, outb.ld);
  };
  NET_OK(conv3(E1A, one_src(n->xin, 0, 32), 0, n->e1a, 0));
  NET_OK(conv3(E1B, one_src(n->e1a, 0, 32), 0, n->c1, 0));
  NET_OK(pool(n->c1, 0, 32, n->p1));
  NET_OK(conv3(E2A, one_src(n->p1, 0, 32), 1, n->e2a, 0));
  NET_OK(conv3(E2B, one_src(n->e2a, 0, 64), 1, n->c2, 0));
  NET_OK(pool(n->c2, 0, 64, n->p2));
  NET_OK(conv3(E3A, one_src(n->p2, 0, 64), 2, n->e3a, 0));
  NET_OK(conv3(E3B, one_src(n->e3a, 0, 128), 2, n->c3, 0));
  NET_OK(pool(n->c3, 0, 128, n->p3));
  NET_OK(conv3(E4A, one_src(n->p3, 0, 128), 3, n->e4a, 0));
  NET_OK(conv3(E4B, one_src(n->e4a, 0, 128), 3, n->e4b, 0));
  NET_OK(conv3(D3A, cat_src(n->c3, 128, n->e4b), 2, n->d3a, 0));
  NET_OK(conv3(D3B, one_src(n->d3a, 0, 128), 2, n->d3b, 0));
  NET_OK(conv3(D2A, cat_src(n->c2, 64, n->d3b), 1, n->d2a, 0));
  NET_OK(conv3(D2B, one_src(n->d2a, 0, 64), 1, n->d2b, 0));
  NET_OK(conv3(D1A, cat_src(n->c1, 32, n->d2b), 0, n->d1a, 0));
  NET_OK(conv3(D1B, one_src(n->d1a, 0, 32), 0, n->d1b, 0));
  const Layer& h = n->L[HEAD];
  NET_OK(conv_launch(n, 1, one_src(n->d1b, 0, 32), h.ci_p, h.Wt,
                     n->master + h.boff, h.co, h.co_p, n->out, true, kOutLd,
                     0, false, B, level_ext(n, Z, H, W, 0)));
  return STML_OK;
}

// Weight and bias gradient of layer li from dPre (ld, off) and its input X.
int layer_wgrad(stml_net* n, int li, const float* dP, int pld, int poff,
                const ConvSrc<bf16>& X, int B, Ext e, const AdamArgs& a,
                bool copy_grad) {
  const Layer& l = n->L[li];
  const int K2 = l.taps;
  const long long P = (long long)B * e.pix();
  const long long nchunks = (P + kWChunk - 1) / kWChunk;
  const int nco = (l.co_p + 63) / 64, nci = (l.ci_p + 63) / 64;
  const int gy = K2 * nco * nci;
  const size_t per_split = (size_t)K2 * l.co_p * l.ci_p;
  long long ns = 1024 / gy;
  if (ns < 1) ns = 1;
  if (ns > nchunks) ns = nchunks;
  if ((size_t)ns * per_split > n->wpart_cap) ns = n->wpart_cap / per_split;
  if (ns < 1) return STML_ENOMEM;
  const long long cps = (nchunks + ns - 1) / ns;
  ns = (nchunks + cps - 1) / cps;
  dim3 grid((unsigned)ns, gy);
#define WGRAD(KK, KZ)                                                     \
  wgrad_kernel<KK, KZ><<<grid, 256, 0, n->stream>>>(                      \
      dP, pld, poff, l.co_p, X, l.ci_p, B, e.z, e.h, e.w, (int)cps, n->wpart)
  if (l.k == 3 && n->dim == 3)
    WGRAD(3, 3);
  else if (l.k == 3)
    WGRAD(3, 1);
  else
    WGRAD(1, 1);
#undef WGRAD
  NET_OK(hipGetLastError());
  const long long pps = (P + kBSplit - 1) / kBSplit;
  const int bs = (int)((P + pps - 1) / pps);
  bias_grad_kernel<<<bs, l.co_p, 0, n->stream>>>(dP, pld, poff, l.co_p, P,
                                                 pps, n->bpart);
  NET_OK(hipGetLastError());
  bias_reduce_kernel<<<l.co, 64, 0, n->stream>>>(n->bpart, bs, l.co_p, n->gb);
  NET_OK(hipGetLastError());
  const int ne = K2 * l.co * l.ci + l.co;
  adam_layer_kernel<<<(ne + 255) / 256, 256, 0, n->stream>>>(
      n->wpart, (int)ns, n->gb, K2, l.co, l.ci, l.co_p, l.ci_p,
      n->master + l.woff, n->m + l.woff, n->v + l.woff,
      copy_grad ? n->grad + l.woff : nullptr, l.Wt, l.Wb, a);
  NET_OK(hipGetLastError());
  return STML_OK;
}

// Backward of a 3x3 conv layer: dPre in place (ReLU mask of its output),
// weight gradient + Adam, and (if dX) the input gradient.  The layer's
// input is in (its first skipC channels) followed, when low is given, by
// the upsampled channels of low.
int conv_back(stml_net* n, int li, Buf& outb, int ooff, const Buf& in,
              float* dX, int dld, int B, int Z, int H, int W,
              const AdamArgs& a, bool copy_grad, const Buf* low = nullptr,
              int skipC = 0) {
  const Layer& l = n->L[li];
  const Ext e = level_ext(n, Z, H, W, in.level);
  const long long P = (long long)B * e.pix();
  relu_bwd_kernel<<<gridsz(P * l.co), 256, 0, n->stream>>>(
      outb.g, outb.ld, ooff, outb.a, outb.ld, ooff, l.co_p, P);
  NET_OK(hipGetLastError());
  // input gradient first: it must use the weights of the forward pass,
  // which the Adam step below replaces
  if (dX)
    NET_OK(conv_launch(n, 3,
                       ConvSrc<float>{outb.g + ooff, outb.ld, 0, nullptr, 0,
                                      0, l.co_p},
                       l.co_p, l.Wb, nullptr, l.ci_p, l.ci_p, dX, true, dld, 0,
                       false, B, e));
  const ConvSrc<bf16> X = low ? cat_src(in, skipC, *low)
                              : one_src(in, 0, l.ci_p);
  return layer_wgrad(n, li, outb.g, outb.ld, ooff, X, B, e, a, copy_grad);
}

}  // namespace

namespace stml {
void net_capacity(const stml_net* n, int* max_batch, long long* max_pixels) {
  *max_batch = n->maxB;
  *max_pixels = ::max_pixels(n);
}
int net_dim(const stml_net* n) { return n->dim; }
}  // namespace stml

// ================================================================ C-ABI

namespace {

// Frame extent of a batch: (H, W) in 2-D, (Z, H, W) in 3-D; every extent a
// multiple of 8 (three poolings), the fastest at most kMaxConvW.
bool parse_ext(int dim, const int* ext, int* Z, int* H, int* W) {
  if (!ext || (dim != 2 && dim != 3)) return false;
  for (int a = 0; a < dim; ++a)
    if (ext[a] < 8 || ext[a] % 8) return false;
  *Z = dim == 3 ? ext[0] : 1;
  *H = ext[dim - 2];
  *W = ext[dim - 1];
  return *W <= kMaxConvW;
}

}  // namespace

extern "C" {

int stml_net_param_count(int dim) {
  if (dim != 2 && dim != 3) return STML_EINVAL;
  int np = 0;
  for (int i = 0; i < kLayers; ++i) {
    const LayerDef d = layer_def(dim, i);
    np += layer_taps(dim, d.k) * d.co * d.ci + d.co;
  }
  return np;
}

size_t stml_net_workspace_bytes(int dim, int max_batch, const int* ext) {
  int Z, H, W;
  if (max_batch < 1 || !parse_ext(dim, ext, &Z, &H, &W)) return 0;
  stml_net tmp;
  tmp.dim = dim;
  tmp.maxB = max_batch;
  tmp.maxZ = Z;
  tmp.maxH = H;
  tmp.maxW = W;
  return net_layout(&tmp, nullptr);
}

int stml_net_create(int dim, int max_batch, const int* ext, void* stream,
                    void* ws, size_t ws_bytes, stml_net** out) {
  if (!out) return STML_EINVAL;
  *out = nullptr;
  size_t need = stml_net_workspace_bytes(dim, max_batch, ext);
  if (!need) return STML_EINVAL;
  if (!ws || ws_bytes < need) return STML_ENOMEM;
  stml_net* n = new stml_net();
  n->dim = dim;
  n->maxB = max_batch;
  parse_ext(dim, ext, &n->maxZ, &n->maxH, &n->maxW);
  n->stream = (hipStream_t)stream;
  net_layout(n, (char*)ws);
  if (hipHostMalloc((void**)&n->htlr, 3 * sizeof(int) * max_frames(n),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&n->hloss, sizeof(double),
                    hipHostMallocDefault) != hipSuccess) {
    stml_net_destroy(n);
    return STML_EDEVICE;
  }
  // zero the whole workspace once: padded weight rows and channels stay 0
  zero_f32_kernel<<<8192, 256, 0, n->stream>>>((float*)ws, need / 4);
  if (hipGetLastError() != hipSuccess ||
      hipStreamSynchronize(n->stream) != hipSuccess) {
    stml_net_destroy(n);
    return STML_EDEVICE;
  }
  *out = n;
  return STML_OK;
}

void stml_net_destroy(stml_net* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  if (n->htlr) (void)hipHostFree(n->htlr);
  if (n->hloss) (void)hipHostFree(n->hloss);
  delete n;
}

int stml_net_set_params(stml_net* n, const float* params) {
  if (!n || !params) return STML_EINVAL;
  NET_OK(hipMemcpyAsync(n->master, params, n->nparam * sizeof(float),
                        hipMemcpyDeviceToDevice, n->stream));
  zero_f32_kernel<<<2048, 256, 0, n->stream>>>(n->m, n->nparam);
  zero_f32_kernel<<<2048, 256, 0, n->stream>>>(n->v, n->nparam);
  for (int i = 0; i < kLayers; ++i) {
    const Layer& l = n->L[i];
    int ne = l.taps * l.co * l.ci;
    weights_from_master_kernel<<<(ne + 255) / 256, 256, 0, n->stream>>>(
        n->master + l.woff, l.taps, l.co, l.ci, l.co_p, l.ci_p, l.Wt, l.Wb);
  }
  n->step = 0;
  NET_OK(hipGetLastError());
  NET_OK(hipStreamSynchronize(n->stream));
  return STML_OK;
}

int stml_net_get_params(const stml_net* n, float* params) {
  if (!n || !params) return STML_EINVAL;
  NET_OK(hipMemcpyAsync(params, n->master, n->nparam * sizeof(float),
                        hipMemcpyDeviceToDevice, n->stream));
  NET_OK(hipStreamSynchronize(n->stream));
  return STML_OK;
}

static int check_shape(const stml_net* n, int B, const int* ext, int* Z,
                       int* H, int* W) {
  if (B < 1 || !parse_ext(n->dim, ext, Z, H, W) ||
      (long long)B * *Z * *H * *W > max_pixels(n))
    return STML_EINVAL;
  return STML_OK;
}

int stml_net_set_input(stml_net* n, const float* x, int C, const float* tgt,
                       int B, const int* ext) {
  if (!n || !x || C < 1 || C > kCinPad) return STML_EINVAL;
  int Z, H, W;
  if (check_shape(n, B, ext, &Z, &H, &W)) return STML_EINVAL;
  const long long N = (long long)Z * H * W, P = (long long)B * N;
  pack_input_kernel<<<gridsz(P * kCinPad), 256, 0, n->stream>>>(x, C, B, N,
                                                                n->xin.a);
  NET_OK(hipGetLastError());
  if (tgt)
    NET_OK(hipMemcpyAsync(n->tgt, tgt, P * n->dim * sizeof(float),
                          hipMemcpyDeviceToDevice, n->stream));
  n->curB = B;
  n->curZ = Z;
  n->curH = H;
  n->curW = W;
  NET_OK(hipStreamSynchronize(n->stream));
  return STML_OK;
}

int stml_net_assemble(stml_net* n, const float* T, const float* U,
                      int n_frames, const int* ext, double h,
                      const int* triples, int B, int with_target) {
  if (!n || !T || !U || !triples || !(h > 0) || n_frames < 3)
    return STML_EINVAL;
  int Z, H, W;
  if (check_shape(n, B, ext, &Z, &H, &W)) return STML_EINVAL;
  for (int b = 0; b < B; ++b) {
    const int t = triples[3 * b], l = triples[3 * b + 1],
              r = triples[3 * b + 2];
    if (!(0 <= l && l < t && t < r && r < n_frames)) return STML_EINVAL;
  }
  for (int i = 0; i < 3 * B; ++i) n->htlr[i] = triples[i];
  NET_OK(hipMemcpyAsync(n->tlr, n->htlr, 3 * B * sizeof(int),
                        hipMemcpyHostToDevice, n->stream));
  const long long N = (long long)Z * H * W;
  assemble_kernel<<<gridsz((long long)B * N), 256, 0, n->stream>>>(
      T, U, n->tlr, B, n->dim, N, 1.0 / h, n->xin.a, n->base,
      with_target ? n->tgt : nullptr);
  NET_OK(hipGetLastError());
  n->curB = B;
  n->curZ = Z;
  n->curH = H;
  n->curW = W;
  NET_OK(hipStreamSynchronize(n->stream));
  return STML_OK;
}

int stml_net_forward(stml_net* n, float* out) {
  if (!n || !n->curB) return STML_ESTATE;
  int rc = net_forward(n, n->curB, n->curZ, n->curH, n->curW);
  if (rc) return rc;
  if (out)
    NET_OK(hipMemcpyAsync(out, n->out,
                          (size_t)n->curB * n->curZ * n->curH * n->curW *
                              kOutLd * sizeof(float),
                          hipMemcpyDeviceToDevice, n->stream));
  NET_OK(hipStreamSynchronize(n->stream));
  return STML_OK;
}

int stml_net_emit(stml_net* n, double h, float* U) {
  if (!n || !n->curB || !U) return STML_ESTATE;
  const long long N = (long long)n->curZ * n->curH * n->curW;
  emit_kernel<<<gridsz((long long)n->curB * N), 256, 0, n->stream>>>(
      n->base, n->out, n->tlr, n->curB, n->dim, N, h, U);
  NET_OK(hipGetLastError());
  NET_OK(hipStreamSynchronize(n->stream));
  return STML_OK;
}

// forward + loss + backward; Adam if lr > 0; gradient copy if grad != NULL
static int net_step(stml_net* n, double lr, float* grad, double* loss) {
  if (!n->curB) return STML_ESTATE;
  const int B = n->curB, Z = n->curZ, H = n->curH, W = n->curW;
  const int dim = n->dim;
  int rc = net_forward(n, B, Z, H, W);
  if (rc) return rc;
  const Ext e0 = level_ext(n, Z, H, W, 0), e1 = level_ext(n, Z, H, W, 1),
            e2 = level_ext(n, Z, H, W, 2), e3 = level_ext(n, Z, H, W, 3);
  const long long P = (long long)B * e0.pix();
  int lb = gridsz(P);
  loss_kernel<<<lb, 256, 0, n->stream>>>(n->out, n->tgt, P, dim, n->dout,
                                         n->lpart);
  loss_final_kernel<<<1, 64, 0, n->stream>>>(n->lpart, lb, n->dloss);
  NET_OK(hipGetLastError());
  AdamArgs a;
  a.apply = lr > 0;
  if (a.apply) n->step += 1;
  a.lr = (float)lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.c1 = a.apply ? (float)(1.0 / (1.0 - std::pow(0.9, n->step))) : 1.f;
  a.c2 = a.apply ? (float)(1.0 / (1.0 - std::pow(0.999, n->step))) : 1.f;
  const bool cg = grad != nullptr;
  hipStream_t s = n->stream;
  // head: dout -> d1b gradient; weight gradient from dout and d1b
  {
    const Layer& l = n->L[HEAD];
    NET_OK(conv_launch(n, 1,
                       ConvSrc<float>{n->dout, kOutLd, 0, nullptr, 0, 0,
                                      l.co_p},
                       l.co_p, l.Wb, nullptr, l.ci_p, l.ci_p, n->d1b.g, true,
                       32, 0, false, B, e0));
    rc = layer_wgrad(n, HEAD, n->dout, kOutLd, 0, one_src(n->d1b, 0, 32), B,
                     e0, a, cg);
    if (rc) return rc;
  }
  // decoder 1
  if ((rc = conv_back(n, D1B, n->d1b, 0, n->d1a, n->d1a.g, 32, B, Z, H, W,
                      a, cg)))
    return rc;
  if ((rc = conv_back(n, D1A, n->d1a, 0, n->c1, n->c1.g, 96, B, Z, H, W, a,
                      cg, &n->d2b, 32)))
    return rc;
  NET_OK(up_bwd_launch(dim, B * e1.pix() * 64, s, (const float*)n->c1.g, 96,
                       32, 64, B, e0.z, e0.h, e0.w, n->d2b.g));
  // decoder 2
  if ((rc = conv_back(n, D2B, n->d2b, 0, n->d2a, n->d2a.g, 64, B, Z, H, W,
                      a, cg)))
    return rc;
  if ((rc = conv_back(n, D2A, n->d2a, 0, n->c2, n->c2.g, 192, B, Z, H, W, a,
                      cg, &n->d3b, 64)))
    return rc;
  NET_OK(up_bwd_launch(dim, B * e2.pix() * 128, s, (const float*)n->c2.g,
                       192, 64, 128, B, e1.z, e1.h, e1.w, n->d3b.g));
  // decoder 3
  if ((rc = conv_back(n, D3B, n->d3b, 0, n->d3a, n->d3a.g, 128, B, Z, H, W,
                      a, cg)))
    return rc;
  if ((rc = conv_back(n, D3A, n->d3a, 0, n->c3, n->c3.g, 256, B, Z, H, W, a,
                      cg, &n->e4b, 128)))
    return rc;
  NET_OK(up_bwd_launch(dim, B * e3.pix() * 128, s, (const float*)n->c3.g,
                       256, 128, 128, B, e2.z, e2.h, e2.w, n->e4b.g));
  // encoder 4 (bottom)
  if ((rc = conv_back(n, E4B, n->e4b, 0, n->e4a, n->e4a.g, 128, B, Z, H, W,
                      a, cg)))
    return rc;
  if ((rc = conv_back(n, E4A, n->e4a, 0, n->p3, n->p3.g, 128, B, Z, H, W, a,
                      cg)))
    return rc;
  NET_OK(pool_bwd_launch(dim, B * e2.pix() * 128, s, (const float*)n->p3.g,
                         128, B, e2.z, e2.h, e2.w, n->c3.g, 256, 0));
  // encoder 3
  if ((rc = conv_back(n, E3B, n->c3, 0, n->e3a, n->e3a.g, 128, B, Z, H, W,
                      a, cg)))
    return rc;
  if ((rc = conv_back(n, E3A, n->e3a, 0, n->p2, n->p2.g, 64, B, Z, H, W, a,
                      cg)))
    return rc;
  NET_OK(pool_bwd_launch(dim, B * e1.pix() * 64, s, (const float*)n->p2.g,
                         64, B, e1.z, e1.h, e1.w, n->c2.g, 192, 0));
  // encoder 2
  if ((rc = conv_back(n, E2B, n->c2, 0, n->e2a, n->e2a.g, 64, B, Z, H, W, a,
                      cg)))
    return rc;
  if ((rc = conv_back(n, E2A, n->e2a, 0, n->p1, n->p1.g, 32, B, Z, H, W, a,
                      cg)))
    return rc;
  NET_OK(pool_bwd_launch(dim, B * e0.pix() * 32, s, (const float*)n->p1.g,
                         32, B, e0.z, e0.h, e0.w, n->c1.g, 96, 0));
  // encoder 1
  if ((rc = conv_back(n, E1B, n->c1, 0, n->e1a, n->e1a.g, 32, B, Z, H, W, a,
                      cg)))
    return rc;
  if ((rc = conv_back(n, E1A, n->e1a, 0, n->xin, nullptr, 0, B, Z, H, W, a,
                      cg)))
    return rc;
  NET_OK(hipGetLastError());
  if (grad)
    NET_OK(hipMemcpyAsync(grad, n->grad, n->nparam * sizeof(float),
                          hipMemcpyDeviceToDevice, n->stream));
  NET_OK(hipMemcpyAsync(n->hloss, n->dloss, sizeof(double),
                        hipMemcpyDeviceToHost, n->stream));
  NET_OK(hipStreamSynchronize(n->stream));
  if (loss) *loss = *n->hloss;
  return STML_OK;
}

int stml_net_gradient(stml_net* n, float* grad, double* loss) {
  if (!n || !grad) return STML_EINVAL;
  return net_step(n, 0.0, grad, loss);
}

int stml_net_train_step(stml_net* n, double lr, double* loss) {
  if (!n || !(lr > 0)) return STML_EINVAL;
  return net_step(n, lr, nullptr, loss);
}

}  // extern "C"
