// Training of a (small) flow network on teacher flows: the distilled student
// of the per-frame path (Sec. 3.2 "Training"; supplementary loss Eq. S2).
//
// Forward: the inference kernels (staging, MFMA convs, fused warp + cost
// volume, head), with every activation kept.  Backward, all FP32:
//   * loss: equally weighted sum over levels of mean (|du| + |dv| + eps)^q
//     against the teacher flow edge-padded, averaged over 2^l x 2^l blocks
//     and divided by 2^l; its gradient seeds d flow_l at every level;
//   * LeakyReLU backward from the stored outputs (slope > 0, so the sign of
//     the output is the sign of the input);
//   * conv data gradient of the stride-1 convs = a stride-1 conv with the
//     weights transposed and flipped, on the MFMA conv kernel; of the
//     stride-2 pyramid convs a gather kernel;
//   * conv weight gradient: a tiled reduction over pixels (vector ALUs,
//     LDS tiles, per-chunk partial sums reduced in a fixed order);
//   * cost volume backward to F1 and to the warped F2; warp backward to the
//     features (scattered with atomics) and to the flow; up2 backward;
//   * AdamW (decoupled weight decay).
// Weights, gradients and Adam moments live in the layout of the weight blob.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/tcflow.h"
#include "act.h"
#include "tc_internal.h"

namespace tc {
namespace {

inline unsigned grid1(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 65535u * 8u) g = 65535u * 8u;
  return (unsigned)(g ? g : 1);
}

// ---------------------------------------------------------------- packing

// Forward packing (the layout of ConvLayer): [cin_pad / kc][9][kc][np],
// packed input channel g <- blob channel cmap[g] (-1: zero).
__global__ void pack_fwd_kernel(const float* __restrict__ blob, int woff, int boff, int cout,
                                int cin, int kc, int cin_pad, int np,
                                const int* __restrict__ cmap, float* __restrict__ w,
                                float* __restrict__ b) {
  const size_t total = (size_t)cin_pad * 9 * np;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int o = (int)(e % np);
    const size_t r = e / np;
    const int kk = (int)(r % kc);
    const int tap = (int)((r / kc) % 9);
    const int chunk = (int)(r / ((size_t)kc * 9));
    const int c = cmap[chunk * kc + kk];
    w[e] = (c >= 0 && o < cout) ? blob[woff + ((size_t)o * cin + c) * 9 + tap] : 0.f;
    if (e < (size_t)np) b[e] = (int)e < cout ? blob[boff + e] : 0.f;
  }
}

// Data-gradient packing: the stride-1 conv from d(output) (cout channels,
// blocks of 8) to d(input) in packed input order, weights
// W'[g][o][2-p][2-q] = W[o][cmap[g]][p][q]; layout [cin'/8][9][8][np'].
__global__ void pack_dgrad_kernel(const float* __restrict__ blob, int woff, int cout, int cin,
                                  int cinp_out, int np_out, const int* __restrict__ cmap,
                                  int cin_pad_f, float* __restrict__ w) {
  const size_t total = (size_t)cinp_out * 9 * np_out;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int g = (int)(e % np_out);
    const size_t r = e / np_out;
    const int o = (int)((r % 8) + (r / (8 * 9)) * 8);
    const int tap = (int)((r / 8) % 9);
    const int c = g < cin_pad_f ? cmap[g] : -1;
    w[e] = (c >= 0 && o < cout) ? blob[woff + ((size_t)o * cin + c) * 9 + (8 - tap)] : 0.f;
  }
}

// F(4x4, 3x3) Winograd weights U = G g G^T of a stride-1 trainer conv, in
// the F(4x4) kernel's layout [32-output slice][chunk of 4 inputs][16-output
// block][lane 16 (input % 4) + output % 16][36 positions] (G: Lavin and
// Gray's F(4x4, 3x3) filter transform, applied in double).  One thread per
// (conv output oc < nout, conv input ic < nin).  Forward: the kernel of blob
// output oc and packed input ic; data gradient (dgrad != 0): conv output =
// packed forward input g = oc, conv input = forward output o = ic, kernel
// flipped.  Entries past the channels are zero.
__global__ void pack_wino4_kernel(const float* __restrict__ blob, int woff, int cout, int cin,
                                  const int* __restrict__ cmap, int cin_pad_f, int dgrad, int nout,
                                  int nin, float* __restrict__ out) {
  const double G[6][3] = {{1.0 / 4, 0.0, 0.0},           {-1.0 / 6, -1.0 / 6, -1.0 / 6},
                          {-1.0 / 6, 1.0 / 6, -1.0 / 6}, {1.0 / 24, 1.0 / 12, 1.0 / 6},
                          {1.0 / 24, -1.0 / 12, 1.0 / 6}, {0.0, 0.0, 1.0}};
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout * nin) return;
  const int oc = e / nin, ic = e % nin;
  const int o = dgrad ? ic : oc, g = dgrad ? oc : ic;
  const int c = g < cin_pad_f ? cmap[g] : -1;
  const bool ok = o < cout && c >= 0;
  double k[9];
  for (int tap = 0; tap < 9; ++tap)
    k[tap] = ok ? (double)blob[woff + ((size_t)o * cin + c) * 9 + (dgrad ? 8 - tap : tap)] : 0.0;
  double Gg[6][3];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 3; ++j) Gg[i][j] = G[i][0] * k[j] + G[i][1] * k[3 + j] + G[i][2] * k[6 + j];
  const int sl = oc / 32, nbk = (oc % 32) / 16, m = oc % 16, chunk = ic / 4, lane = 16 * (ic % 4) + m;
  float* dst = out + ((((size_t)sl * (nin / 4) + chunk) * 2 + nbk) * 64 + lane) * 36;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j)
      dst[6 * i + j] = (float)(Gg[i][0] * G[j][0] + Gg[i][1] * G[j][1] + Gg[i][2] * G[j][2]);
}

// ---------------------------------------------------------------- elementwise

// dst (blocks [cb_d, cb_d + nb) of a cbt_d-block buffer) =
//   (dst + add) * lrelu'(y), add and y with their own block offsets
__global__ void lrelu_bwd_kernel(float* __restrict__ dst, int cbt_d, int cb_d,
                                 const float* __restrict__ add, int cbt_a, int cb_a,
                                 const float* __restrict__ y, int cbt_y, int cb_y, int nb, int n,
                                 int P, float slope) {
  const size_t total = (size_t)n * nb * P * 2;  // float4 units
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int half = (int)(e & 1);
    const size_t r = e >> 1;
    const int p = (int)(r % P);
    const int b = (int)((r / P) % nb);
    const int img = (int)(r / ((size_t)P * nb));
    f4* d = reinterpret_cast<f4*>(dst + (((size_t)img * cbt_d + cb_d + b) * P + p) * 8) + half;
    const f4 yv = *(reinterpret_cast<const f4*>(y + (((size_t)img * cbt_y + cb_y + b) * P + p) * 8) + half);
    f4 v = *d;
    if (add) v += *(reinterpret_cast<const f4*>(add + (((size_t)img * cbt_a + cb_a + b) * P + p) * 8) + half);
    v.x *= yv.x >= 0.f ? 1.f : slope;
    v.y *= yv.y >= 0.f ? 1.f : slope;
    v.z *= yv.z >= 0.f ? 1.f : slope;
    v.w *= yv.w >= 0.f ? 1.f : slope;
    *d = v;
  }
}

__global__ void zero_kernel(float* __restrict__ p, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = 0.f;
}

// ---------------------------------------------------------------- loss

// Per level-l pixel: target = mean of the edge-padded teacher over the
// 2^l x 2^l block / 2^l; e = flow - target; r = |e_u| + |e_v| + eps;
// loss r^q, d flow = scale q r^(q-1) sign(e) into a one-block buffer.
// One partial sum per workgroup.
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ flow,
                                                   const float* __restrict__ T, int n, int H,
                                                   int W, int hl, int wl, int s, float eps,
                                                   float q, float scale, float* __restrict__ dflow,
                                                   float* __restrict__ partial) {
  __shared__ float red[256];
  const size_t P = (size_t)hl * wl;
  const size_t total = (size_t)n * P;
  float acc = 0.f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int img = (int)(i / P);
    const int p = (int)(i - (size_t)img * P);
    const int y = p / wl, x = p - (p / wl) * wl;
    float tu = 0.f, tv = 0.f;
    for (int dy = 0; dy < s; ++dy) {
      const int yy = min(y * s + dy, H - 1);
      for (int dx = 0; dx < s; ++dx) {
        const int xx = min(x * s + dx, W - 1);
        tu += T[((size_t)img * 2 + 0) * H * W + (size_t)yy * W + xx];
        tv += T[((size_t)img * 2 + 1) * H * W + (size_t)yy * W + xx];
      }
    }
    const float inv = 1.f / ((float)s * s * s);
    tu *= inv;
    tv *= inv;
    const float2 f = reinterpret_cast<const float2*>(flow)[i];
    const float eu = f.x - tu, ev = f.y - tv;
    const float r = fabsf(eu) + fabsf(ev) + eps;
    const float rq = powf(r, q);
    acc += rq;
    const float gq = scale * q * rq / r;
    const float su = eu > 0.f ? 1.f : (eu < 0.f ? -1.f : 0.f);
    const float sv = ev > 0.f ? 1.f : (ev < 0.f ? -1.f : 0.f);
    f4* o = reinterpret_cast<f4*>(dflow + i * 8);
    o[0] = f4{gq * su, gq * sv, 0.f, 0.f};
    o[1] = f4{0.f, 0.f, 0.f, 0.f};
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] * scale;
}

// loss = sum of the partial sums in index order (one workgroup)
__global__ __launch_bounds__(256) void sum_kernel(const float* __restrict__ partial, int n,
                                                  float* __restrict__ out) {
  __shared__ float red[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ---------------------------------------------------------------- weight gradient
//
// dW[o][g][tap] = sum over images and output pixels of dz[o](y, x) *
// X[g](s y + p - 1, s x + q - 1) (zero outside), per pixel chunk as partial
// sums, then added over the chunks in a fixed order.
struct WgArgs {
  const float* dz;  // blocked, dz_cbt blocks per image, first block dz_cb0
  int dz_cbt, dz_cb0;
  const float* x0;  // input view 0: blocks [0, nb0) of the packed input
  int x0_cbt, x0_cb0, nb0;
  const float* x1;  // input view 1: blocks [nb0, ...)
  int x1_cbt, x1_cb0;
  int n, ho, wo, hi, wi, stride;
  int nob, ncb, chunks;
  float* partial;   // [chunk][ob][cb][8][KB][9]
};

constexpr int WG_TW = 64;

// The chunk sums on the FP32 matrix cores (v_mfma_f32_16x16x4_f32), as a GEMM
// with M = output channels (MB blocks of 16), N = (tap, input channel) and
// K = output pixels: N block j is tap j = 3 p + q, its column n input
// channel 16 cg + n of the workgroup's 16-channel group cg.  A workgroup owns
// a range of row tiles (64 output pixels of one row), one channel group and
// one group of MB output blocks (output channels 16 MB mg ...);
// per tile it stages dz [64][16 MB] and the three input rows [3][cols][16] in
// LDS (pitches chosen so a K step's 64 lanes read distinct banks), and wave w
// takes K steps w, w + 4, w + 8, w + 12 (4 pixels each): one A read and nine
// B reads feed 9 MB matrix instructions.  At the end the four waves' sums
// are added in wave order and written as the chunk's partials
// ([chunk][ob][cb][8][KB][9]).
template <int MB, int S>
__global__ __launch_bounds__(256, 2) void wgrad_mfma_kernel(WgArgs a, int KB, int cout, int cin_pad) {
  constexpr int TW = WG_TW;
  constexpr int PO = 32 * MB - 16;          // dz floats per pixel (16 mod 32)
  constexpr int XWM = S * (TW - 1) + 3;     // input columns
  constexpr int PC = 16;                    // input floats per staged pixel
  constexpr int NDZ = TW * PO, NX = 3 * XWM * PC;
  constexpr int RDZ = TW * 2 * MB * 2 / 256;         // dz float4 per thread and tile
  constexpr int RX = (3 * XWM * 4 + 255) / 256;      // input float4 per thread and tile
  static_assert(TW * 2 * MB * 2 % 256 == 0, "dz tile split");
  constexpr int SMEM = NDZ + NX > 3 * 9 * 256 ? NDZ + NX : 3 * 9 * 256;  // staging, or the wave reduction
  __shared__ __attribute__((aligned(16))) float smem[SMEM];
  float* const sdz = smem;
  float* const sx = smem + NDZ;

  const int cg = blockIdx.y;
  const int obase = 16 * MB * blockIdx.z;  // first output channel of the group
  const int ob0 = obase / 8, nobg = min(2 * MB, a.nob - ob0);
  const int xt = (a.wo + TW - 1) / TW;
  const long tiles = (long)a.n * a.ho * xt;
  const long per = (tiles + a.chunks - 1) / a.chunks;
  const long t0 = blockIdx.x * per, t1 = min(tiles, t0 + per);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kg = lane >> 4, ln = lane & 15;
  const size_t Pi = (size_t)a.hi * a.wi, Po = (size_t)a.ho * a.wo;

  f4 acc[MB][9];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[m][j] = f4{0.f, 0.f, 0.f, 0.f};

  // A tile's loads go to registers one tile ahead (rdz: 64 pixels x the
  // group's blocks x 2 halves of 4 output channels; rx: 3 input rows x
  // XWM columns x 4 quarters of the 16 channels), zero outside the image,
  // past the output channels and past the packed input channels.
  f4 rdz[RDZ], rx[RX];
  auto load = [&](long t) {
    const int img = (int)(t / ((long)a.ho * xt));
    const int rem = (int)(t - (long)img * a.ho * xt);
    const int yo = rem / xt, x0 = (rem % xt) * TW;
#pragma unroll
    for (int j = 0; j < RDZ; ++j) {
      const int e = tid + 256 * j;
      const int h = e & 1, px = (e >> 1) % TW, obl = (e >> 1) / TW;
      const int xo = x0 + px, o = obase + obl * 8 + 4 * h;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (obl < nobg && xo < a.wo)
        v = *(reinterpret_cast<const f4*>(a.dz + (((size_t)img * a.dz_cbt + a.dz_cb0 + ob0 + obl) * Po +
                                                  (size_t)yo * a.wo + xo) *
                                                     8) +
              h);
      if (o + 0 >= cout) v.x = 0.f;
      if (o + 1 >= cout) v.y = 0.f;
      if (o + 2 >= cout) v.z = 0.f;
      if (o + 3 >= cout) v.w = 0.f;
      rdz[j] = v;
    }
#pragma unroll
    for (int j = 0; j < RX; ++j) {
      const int e = tid + 256 * j;
      const int q4 = e & 3, col = (e >> 2) % XWM, row = (e >> 2) / XWM;
      const int yi = S * yo + row - 1, xi = S * x0 + col - 1;
      const int g = cg * 16 + q4 * 4;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (row < 3 && g < cin_pad && yi >= 0 && yi < a.hi && xi >= 0 && xi < a.wi) {
        const int b = g / KB, off = g - b * KB;
        const float* xb;
        int xcbt, xblk;
        if (b < a.nb0) {
          xb = a.x0; xcbt = a.x0_cbt; xblk = a.x0_cb0 + b;
        } else {
          xb = a.x1; xcbt = a.x1_cbt; xblk = a.x1_cb0 + b - a.nb0;
        }
        v = *reinterpret_cast<const f4*>(xb + (((size_t)img * xcbt + xblk) * Pi + (size_t)yi * a.wi + xi) * KB +
                                         off);
      }
      rx[j] = v;
    }
  };

  if (t0 < t1) load(t0);
  for (long t = t0; t < t1; ++t) {
#pragma unroll
    for (int j = 0; j < RDZ; ++j) {
      const int e = tid + 256 * j;
      const int h = e & 1, px = (e >> 1) % TW, obl = (e >> 1) / TW;
      *reinterpret_cast<f4*>(sdz + px * PO + obl * 8 + 4 * h) = rdz[j];
    }
#pragma unroll
    for (int j = 0; j < RX; ++j) {
      const int e = tid + 256 * j;
      const int q4 = e & 3, col = (e >> 2) % XWM, row = (e >> 2) / XWM;
      if (row < 3) *reinterpret_cast<f4*>(sx + (row * XWM + col) * PC + q4 * 4) = rx[j];
    }
    __syncthreads();
    if (t + 1 < t1) load(t + 1);
#pragma unroll
    for (int i = 0; i < TW / 16; ++i) {
      const int px = 4 * (wave + 4 * i) + kg;  // this lane's pixel (K index)
      float av[MB];
#pragma unroll
      for (int m = 0; m < MB; ++m) av[m] = sdz[px * PO + m * 16 + ln];
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const float bv = sx[((j / 3) * XWM + S * px + j % 3) * PC + ln];
#pragma unroll
        for (int m = 0; m < MB; ++m) acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m], bv, acc[m][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // add the waves' sums in wave order; D[m = 4 kg + v][n = ln] of block
  // (mb, j) is output channel obase + 16 mb + 4 kg + v, input channel
  // 16 cg + ln, tap j
  float* out = a.partial + (size_t)blockIdx.x * a.nob * 8 * cin_pad * 9;
  float* red = smem;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    if (wave > 0)
#pragma unroll
      for (int j = 0; j < 9; ++j) *reinterpret_cast<f4*>(red + ((wave - 1) * 9 + j) * 256 + lane * 4) = acc[m][j];
    __syncthreads();
    if (wave == 0) {
      const int g = cg * 16 + ln;
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        f4 v = acc[m][j];
#pragma unroll
        for (int w = 0; w < 3; ++w) {
          const f4 r = *reinterpret_cast<const f4*>(red + (w * 9 + j) * 256 + lane * 4);
          v.x += r.x;
          v.y += r.y;
          v.z += r.z;
          v.w += r.w;
        }
        const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int o = obase + 16 * m + 4 * kg + k;
          if (o < 8 * a.nob && g < cin_pad) {
            const int cb = g / KB, gg = g - cb * KB;
            out[(((size_t)(o / 8) * a.ncb + cb) * 8 + o % 8) * KB * 9 + gg * 9 + j] = vv[k];
          }
        }
      }
    }
    __syncthreads();
  }
}

// grad[woff + (o cin + cmap[g]) 9 + tap] = sum over chunks of the partials.
// A workgroup takes 64 consecutive partial entries (lane = entry, so every
// chunk's read is one contiguous 256-byte row); wave w adds chunks
// [w per, (w + 1) per) in order, and wave 0 adds the four sums in wave order.
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float* __restrict__ partial, int chunks,
                                                           int nob, int ncb, int KB, int cout, int cin,
                                                           int cin_pad, const int* __restrict__ cmap,
                                                           float* __restrict__ grad, int woff) {
  __shared__ float red[3][64];
  const int per_chunk = nob * ncb * 8 * KB * 9;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int per = (chunks + 3) / 4, k0 = wave * per, k1 = min(chunks, k0 + per);
  float sum = 0.f;
  if (e < per_chunk) {
    const float* src = partial + e;
    int k = k0;
    for (; k + 4 <= k1; k += 4) {
      const float v0 = src[(size_t)k * per_chunk], v1 = src[(size_t)(k + 1) * per_chunk];
      const float v2 = src[(size_t)(k + 2) * per_chunk], v3 = src[(size_t)(k + 3) * per_chunk];
      sum = (((sum + v0) + v1) + v2) + v3;
    }
    for (; k < k1; ++k) sum += src[(size_t)k * per_chunk];
  }
  if (wave > 0) red[wave - 1][lane] = sum;
  __syncthreads();
  if (wave > 0 || e >= per_chunk) return;
  sum = ((sum + red[0][lane]) + red[1][lane]) + red[2][lane];
  // entry e = (((ob ncb + cb) 8 + oo) KB + gg) 9 + tap
  const int tap = e % 9, gg = (e / 9) % KB, oo = (e / (9 * KB)) % 8, cb = (e / (72 * KB)) % ncb;
  const int ob = e / (72 * KB * ncb);
  const int o = ob * 8 + oo, g = cb * KB + gg;
  if (o >= cout || g >= cin_pad) return;
  const int c = cmap[g];
  if (c < 0) return;
  grad[woff + ((size_t)o * cin + c) * 9 + tap] = sum;
}

// bias gradient: per (chunk, output channel) partial sums of dz, then a
// fixed-order reduction
__global__ __launch_bounds__(256) void bgrad_kernel(const float* __restrict__ dz, int cbt, int cb0,
                                                    int nob, int n, int P, int chunks,
                                                    float* __restrict__ partial) {
  __shared__ float red[256][9];
  const int ob = blockIdx.y;
  const size_t total = (size_t)n * P;
  const size_t per = (total + chunks - 1) / chunks;
  const size_t i0 = blockIdx.x * per, i1 = min(total, i0 + per);
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (size_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const size_t img = i / P, p = i - img * P;
    float v[8];
    load8(dz + ((img * cbt + cb0 + ob) * P + p) * 8, v);
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] += v[k];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
#pragma unroll
      for (int k = 0; k < 8; ++k) red[threadIdx.x][k] += red[threadIdx.x + st][k];
    __syncthreads();
  }
  if (threadIdx.x < 8) partial[((size_t)blockIdx.x * nob + ob) * 8 + threadIdx.x] = red[0][threadIdx.x];
}

// one workgroup per output channel: thread k adds chunks k, k + 256, ... in
// order, then a fixed-order tree over the 256 sums
__global__ __launch_bounds__(256) void bgrad_reduce_kernel(const float* __restrict__ partial, int chunks,
                                                           int nob, int cout, float* __restrict__ grad,
                                                           int boff) {
  __shared__ float red[256];
  const int o = blockIdx.x;
  float sum = 0.f;
  for (int k = threadIdx.x; k < chunks; k += 256) sum += partial[((size_t)k * nob + o / 8) * 8 + o % 8];
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0 && o < cout) grad[boff + o] = red[0];
}

// ---------------------------------------------------------------- stride-2 data gradient
//
// dX[c](yi, xi) += sum_o sum_{p,q} W[o][c][p][q] dz[o]((yi + 1 - p) / 2,
// (xi + 1 - q) / 2) over the taps whose output position is integral and in
// range.  One thread per (image, input pixel, block of 8 input channels);
// the layer's weights for that block in LDS.
__global__ __launch_bounds__(256) void dgrad_s2_kernel(const float* __restrict__ dz, int ob_n,
                                                       const float* __restrict__ blob, int woff,
                                                       int cout, int cin, float* __restrict__ dx,
                                                       int n, int hi, int wi, int ho, int wo) {
  __shared__ float sw[128 * 8 * 9];  // [o][c 8][tap]
  const int cb = blockIdx.y;
  for (int e = threadIdx.x; e < cout * 8 * 9; e += 256) {
    const int tap = e % 9, c = (e / 9) % 8, o = e / 72;
    const int cc = cb * 8 + c;
    sw[e] = cc < cin ? blob[woff + ((size_t)o * cin + cc) * 9 + tap] : 0.f;
  }
  __syncthreads();
  const size_t Pi = (size_t)hi * wi, Po = (size_t)ho * wo;
  const size_t total = (size_t)n * Pi;
  const int cbt_x = (cin + 7) / 8;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int img = (int)(i / Pi);
    const int pix = (int)(i - (size_t)img * Pi);
    const int yi = pix / wi, xi = pix - (pix / wi) * wi;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int p = 0; p < 3; ++p) {
      const int ty = yi + 1 - p;
      if (ty < 0 || (ty & 1) || (ty >> 1) >= ho) continue;
      for (int q = 0; q < 3; ++q) {
        const int tx = xi + 1 - q;
        if (tx < 0 || (tx & 1) || (tx >> 1) >= wo) continue;
        const size_t po = (size_t)(ty >> 1) * wo + (tx >> 1);
        const int tap = 3 * p + q;
        for (int o = 0; o < cout; ++o) {
          const float d = dz[(((size_t)img * ob_n + o / 8) * Po + po) * 8 + o % 8];
#pragma unroll
          for (int c = 0; c < 8; ++c) acc[c] += d * sw[(o * 8 + c) * 9 + tap];
        }
      }
    }
    float* dst = dx + (((size_t)img * cbt_x + cb) * Pi + pix) * 8;
    float v[8];
    load8(dst, v);
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] += acc[c];
    store8(dst, v);
  }
}

// ---------------------------------------------------------------- warp and cost volume

struct Taps {
  int x0, y0;
  float ax, ay;
};
__device__ inline Taps taps_of(int x, int y, float fx, float fy) {
  const float sx = (float)x + fx, sy = (float)y + fy;
  const float bx = floorf(sx), by = floorf(sy);
  return Taps{(int)bx, (int)by, sx - bx, sy - by};
}

// F2w (n images, nb blocks) = bilinear zero-padded warp of F2 by U (compact
// float2, or null for zero flow)
__global__ void warp_kernel(const float* __restrict__ F2, const float* __restrict__ U, int n,
                            int nb, int h, int w, float* __restrict__ out) {
  const size_t P = (size_t)h * w;
  const size_t total = (size_t)n * P;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int img = (int)(i / P);
    const int pix = (int)(i - (size_t)img * P);
    const int y = pix / w, x = pix - (pix / w) * w;
    const float2 u = U ? reinterpret_cast<const float2*>(U)[i] : make_float2(0.f, 0.f);
    const Taps t = taps_of(x, y, u.x, u.y);
    for (int b = 0; b < nb; ++b) {
      float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      const float* base = F2 + ((size_t)img * nb + b) * P * 8;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int xi = t.x0 + (k & 1), yi = t.y0 + (k >> 1);
        if (xi < 0 || xi >= w || yi < 0 || yi >= h) continue;
        const float wt = ((k & 1) ? t.ax : 1.f - t.ax) * ((k >> 1) ? t.ay : 1.f - t.ay);
        float v[8];
        load8(base + ((size_t)yi * w + xi) * 8, v);
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] += wt * v[c];
      }
      store8(out + (((size_t)img * nb + b) * P + pix) * 8, acc);
    }
  }
}

// dF1(x) += dZ[F1](x) + sum_k g_k(x) F2w(x + d_k), with g_k = dZ[cv_k] times
// the LeakyReLU slope at Z[cv_k] and 1 / C (the cost volume's mean over the
// channels, Sec. 3.2 correlation), formed where it is read.  A workgroup owns a
// 16 x 16 pixel tile: each pixel's 81 g_k sit in registers, and each 8-channel
// block's F2w over the tile and its 4-pixel halo is staged in LDS (zero
// outside the image, which drops the out-of-image displacements).
constexpr int CV_R = 4, CV_T = 16, CV_H = CV_T + 2 * CV_R, CV_NK = (2 * CV_R + 1) * (2 * CV_R + 1);

__global__ __launch_bounds__(256) void cv_bwd_f1_kernel(const float* __restrict__ dZ, int dz_cbt, int cv_cb0,
                                                        const float* __restrict__ Z, int zcb, float slope,
                                                        float invC, const float* __restrict__ F2w, int nb,
                                                        int n, int h, int w, float* __restrict__ dF1) {
  __shared__ f4 sf[CV_H * CV_H * 2];  // [position][two halves of the block]
  const int tx = threadIdx.x & (CV_T - 1), ty = threadIdx.x / CV_T;
  const int x0 = blockIdx.x * CV_T, y0 = blockIdx.y * CV_T, img = blockIdx.z;
  const int x = x0 + tx, y = y0 + ty;
  const bool in = x < w && y < h;
  const size_t P = (size_t)h * w;
  const int pix = in ? y * w + x : 0;
  float g[CV_NK];
  {
    const float* gb = dZ + ((size_t)img * dz_cbt + cv_cb0) * P * 8 + (size_t)pix * 8;
    const float* zb = Z + (size_t)img * zcb * P * 8 + (size_t)pix * 8;
#pragma unroll
    for (int kb = 0; kb < (CV_NK + 7) / 8; ++kb) {
      float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (in) {
        load8(gb + (size_t)kb * P * 8, v);
        load8(zb + (size_t)kb * P * 8, z);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (kb * 8 + c < CV_NK) g[kb * 8 + c] = v[c] * (z[c] >= 0.f ? invC : slope * invC);
    }
  }
  for (int b = 0; b < nb; ++b) {
    const float* fb = F2w + ((size_t)img * nb + b) * P * 8;
    __syncthreads();
    for (int e = threadIdx.x; e < CV_H * CV_H * 2; e += 256) {
      const int hf = e & 1, pos = e >> 1;
      const int yy = y0 - CV_R + pos / CV_H, xx = x0 - CV_R + pos % CV_H;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (yy >= 0 && yy < h && xx >= 0 && xx < w) v = ldg(reinterpret_cast<const f4*>(fb + ((size_t)yy * w + xx) * 8) + hf);
      sf[e] = v;
    }
    __syncthreads();
    if (!in) continue;
    float acc[8];
    load8(dZ + (((size_t)img * dz_cbt + b) * P + pix) * 8, acc);
#pragma unroll
    for (int k = 0; k < CV_NK; ++k) {
      const int dy = k / (2 * CV_R + 1), dx = k % (2 * CV_R + 1);
      const int pos = (ty + dy) * CV_H + tx + dx;
      const f4 a0 = sf[2 * pos], a1 = sf[2 * pos + 1];
      acc[0] += g[k] * a0.x;
      acc[1] += g[k] * a0.y;
      acc[2] += g[k] * a0.z;
      acc[3] += g[k] * a0.w;
      acc[4] += g[k] * a1.x;
      acc[5] += g[k] * a1.y;
      acc[6] += g[k] * a1.z;
      acc[7] += g[k] * a1.w;
    }
    float* dst = dF1 + (((size_t)img * nb + b) * P + pix) * 8;
    float cur[8];
    load8(dst, cur);
#pragma unroll
    for (int c = 0; c < 8; ++c) cur[c] += acc[c];
    store8(dst, cur);
  }
}

// dF2w(y) = sum_k g_k(y - d_k) F1(y - d_k), g_k as above.  A workgroup owns a 16 x 16
// pixel tile; per 8-channel block of F1 it stages F1 over the tile and its
// 4-pixel halo in LDS, then, one block of 8 displacements at a time, the
// displacements' g over the same window (both zero outside the image, which
// drops the out-of-image sources), and gathers.
__global__ __launch_bounds__(256) void cv_bwd_f2w_kernel(const float* __restrict__ dZ, int dz_cbt, int cv_cb0,
                                                         const float* __restrict__ Z, int zcb, float slope,
                                                         float invC, const float* __restrict__ F1, int nb,
                                                         int n, int h, int w, float* __restrict__ dF2w) {
  __shared__ f4 sf[CV_H * CV_H * 2];       // F1 block: [position][two halves]
  __shared__ float sg[CV_H * CV_H * 8];    // g of 8 displacements: [position][8]
  const int tx = threadIdx.x & (CV_T - 1), ty = threadIdx.x / CV_T;
  const int x0 = blockIdx.x * CV_T, y0 = blockIdx.y * CV_T, img = blockIdx.z;
  const int x = x0 + tx, y = y0 + ty;
  const bool in = x < w && y < h;
  const size_t P = (size_t)h * w;
  const float* gbase = dZ + ((size_t)img * dz_cbt + cv_cb0) * P * 8;
  const float* zbase = Z + (size_t)img * zcb * P * 8;
  for (int b = 0; b < nb; ++b) {
    const float* fb = F1 + ((size_t)img * nb + b) * P * 8;
    __syncthreads();
    for (int e = threadIdx.x; e < CV_H * CV_H * 2; e += 256) {
      const int hf = e & 1, pos = e >> 1;
      const int yy = y0 - CV_R + pos / CV_H, xx = x0 - CV_R + pos % CV_H;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (yy >= 0 && yy < h && xx >= 0 && xx < w) v = ldg(reinterpret_cast<const f4*>(fb + ((size_t)yy * w + xx) * 8) + hf);
      sf[e] = v;
    }
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < (CV_NK + 7) / 8; ++kb) {
      __syncthreads();
      for (int e = threadIdx.x; e < CV_H * CV_H * 2; e += 256) {
        const int hf = e & 1, pos = e >> 1;
        const int yy = y0 - CV_R + pos / CV_H, xx = x0 - CV_R + pos % CV_H;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (yy >= 0 && yy < h && xx >= 0 && xx < w) {
          const size_t q = ((size_t)kb * P + (size_t)yy * w + xx) * 8;
          const f4 d = ldg(reinterpret_cast<const f4*>(gbase + q) + hf);
          const f4 z = ldg(reinterpret_cast<const f4*>(zbase + q) + hf);
          v.x = d.x * (z.x >= 0.f ? invC : slope * invC);
          v.y = d.y * (z.y >= 0.f ? invC : slope * invC);
          v.z = d.z * (z.z >= 0.f ? invC : slope * invC);
          v.w = d.w * (z.w >= 0.f ? invC : slope * invC);
        }
        *reinterpret_cast<f4*>(sg + pos * 8 + hf * 4) = v;
      }
      __syncthreads();
      if (!in) continue;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = kb * 8 + j;
        if (k >= CV_NK) break;
        // source y - d_k with d_k = (k / 9 - 4, k % 9 - 4), in window coordinates
        const int pos = (ty + 2 * CV_R - k / (2 * CV_R + 1)) * CV_H + tx + 2 * CV_R - k % (2 * CV_R + 1);
        const float gv = sg[pos * 8 + j];
        const f4 a0 = sf[2 * pos], a1 = sf[2 * pos + 1];
        acc[0] += gv * a0.x;
        acc[1] += gv * a0.y;
        acc[2] += gv * a0.z;
        acc[3] += gv * a0.w;
        acc[4] += gv * a1.x;
        acc[5] += gv * a1.y;
        acc[6] += gv * a1.z;
        acc[7] += gv * a1.w;
      }
    }
    if (in) store8(dF2w + (((size_t)img * nb + b) * P + (size_t)y * w + x) * 8, acc);
  }
}

// Warp backward: dF2 (scattered) and
// dU = dZ[U] + dflow + sum_c dF2w_c d F2w_c / dU  (U null: zero flow and no
// dU).  A workgroup owns a 16 x 16 pixel tile.  The in-image bilinear taps of
// its pixels span a window of the source image; when the window has at most
// WB_WIN positions, each 8-channel block's tap contributions are first added
// in LDS (LDS atomics), and the window is then added to dF2 with one global
// atomic per nonzero entry: about 9 global atomics per pixel and block for a
// smooth flow instead of 32.  Wider windows scatter straight to dF2.
constexpr int WB_T = 16, WB_WIN = 40 * 40;

__global__ __launch_bounds__(256) void warp_bwd_kernel(const float* __restrict__ dF2w, const float* __restrict__ F2,
                                                       const float* __restrict__ U, int n, int nb, int h, int w,
                                                       float* __restrict__ dF2, const float* __restrict__ dZ,
                                                       int dz_cbt, int u_cb, int u_c,
                                                       const float* __restrict__ dflow, float* __restrict__ dU) {
  __shared__ float win[WB_WIN * 8];
  __shared__ int bb[4];  // window: x min, x max, y min, y max
  const int x = blockIdx.x * WB_T + (threadIdx.x & 15), y = blockIdx.y * WB_T + (threadIdx.x >> 4);
  const int img = blockIdx.z;
  const bool in = x < w && y < h;
  const size_t P = (size_t)h * w;
  const int pix = in ? y * w + x : 0;
  const size_t i = (size_t)img * P + pix;
  const float2 u = in && U ? reinterpret_cast<const float2*>(U)[i] : make_float2(0.f, 0.f);
  const Taps t = taps_of(x, y, u.x, u.y);
  if (threadIdx.x == 0) {
    bb[0] = w;
    bb[1] = -1;
    bb[2] = h;
    bb[3] = -1;
  }
  __syncthreads();
  if (in) {
    atomicMin(&bb[0], max(t.x0, 0));
    atomicMax(&bb[1], min(t.x0 + 1, w - 1));
    atomicMin(&bb[2], max(t.y0, 0));
    atomicMax(&bb[3], min(t.y0 + 1, h - 1));
  }
  __syncthreads();
  const int wx0 = bb[0], wy0 = bb[2];
  const int ww = bb[1] - wx0 + 1, wh = bb[3] - wy0 + 1;
  const bool agg = ww > 0 && wh > 0 && ww * wh <= WB_WIN;
  const int nwin = agg ? ww * wh * 8 : 0;

  float gx = 0.f, gy = 0.f;
  for (int b = 0; b < nb; ++b) {
    const float* fb = F2 + ((size_t)img * nb + b) * P * 8;
    float* db = dF2 + ((size_t)img * nb + b) * P * 8;
    for (int e = threadIdx.x; e < nwin; e += 256) win[e] = 0.f;
    if (agg) __syncthreads();
    if (in) {
      float g[8];
      load8(dF2w + (((size_t)img * nb + b) * P + pix) * 8, g);
      float F[4][8];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int xi = t.x0 + (k & 1), yi = t.y0 + (k >> 1);
        const bool ok = xi >= 0 && xi < w && yi >= 0 && yi < h;
        if (ok) {
          load8(fb + ((size_t)yi * w + xi) * 8, F[k]);
          const float wt = ((k & 1) ? t.ax : 1.f - t.ax) * ((k >> 1) ? t.ay : 1.f - t.ay);
          if (wt != 0.f) {
            if (agg) {
              float* d = win + ((yi - wy0) * ww + (xi - wx0)) * 8;
#pragma unroll
              for (int c = 0; c < 8; ++c)
                if (g[c] != 0.f) atomicAdd(d + c, wt * g[c]);
            } else {
              float* d = db + ((size_t)yi * w + xi) * 8;
#pragma unroll
              for (int c = 0; c < 8; ++c)
                if (g[c] != 0.f) unsafeAtomicAdd(d + c, wt * g[c]);
            }
          }
        } else {
#pragma unroll
          for (int c = 0; c < 8; ++c) F[k][c] = 0.f;
        }
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        // d/dsx: (1 - ay)(F01 - F00) + ay (F11 - F10); d/dsy: (1 - ax)(F10 - F00) + ax (F11 - F01)
        gx += g[c] * ((1.f - t.ay) * (F[1][c] - F[0][c]) + t.ay * (F[3][c] - F[2][c]));
        gy += g[c] * ((1.f - t.ax) * (F[2][c] - F[0][c]) + t.ax * (F[3][c] - F[1][c]));
      }
    }
    if (agg) {
      __syncthreads();
      for (int e = threadIdx.x; e < nwin; e += 256) {
        const float v = win[e];
        if (v != 0.f) {
          const int pos = e >> 3, c = e & 7;
          const int yy = wy0 + pos / ww, xx = wx0 + pos % ww;
          unsafeAtomicAdd(db + ((size_t)yy * w + xx) * 8 + c, v);
        }
      }
      __syncthreads();
    }
  }
  if (in && dU) {
    const float* zu = dZ + (((size_t)img * dz_cbt + u_cb) * P + pix) * 8;
    const float* df = dflow + i * 8;
    reinterpret_cast<float2*>(dU)[i] = make_float2(gx + zu[u_c] + df[0], gy + zu[u_c + 1] + df[1]);
  }
}

// d flow_{l+1} (one-block buffer, channels 0, 1) += 2 up2^T(dU): a coarse
// pixel gathers the fine pixels whose bilinear taps use it.
__device__ inline void up_tap(int i, int n, int& i0, int& i1, float& f) {
  float src = fmaxf((i + 0.5f) * 0.5f - 0.5f, 0.f);
  i0 = min((int)src, n - 1);
  f = src - (float)i0;
  if (i0 >= n - 1) f = 0.f;
  i1 = min(i0 + 1, n - 1);
}

__global__ void up2_bwd_kernel(const float* __restrict__ dU, int n, int h, int w,
                               float* __restrict__ dflow) {
  const size_t P = (size_t)h * w;
  const size_t total = (size_t)n * P;
  const int H = 2 * h, W = 2 * w;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int img = (int)(i / P);
    const int pix = (int)(i - (size_t)img * P);
    const int Y = pix / w, X = pix - (pix / w) * w;
    float su = 0.f, sv = 0.f;
    for (int fy = 2 * Y - 1; fy <= 2 * Y + 2; ++fy) {
      if (fy < 0 || fy >= H) continue;
      int r0, r1;
      float ry;
      up_tap(fy, h, r0, r1, ry);
      const float wy = (r0 == Y ? 1.f - ry : 0.f) + (r1 == Y ? ry : 0.f);
      if (wy == 0.f) continue;
      for (int fx = 2 * X - 1; fx <= 2 * X + 2; ++fx) {
        if (fx < 0 || fx >= W) continue;
        int c0, c1;
        float rx;
        up_tap(fx, w, c0, c1, rx);
        const float wx = (c0 == X ? 1.f - rx : 0.f) + (c1 == X ? rx : 0.f);
        if (wx == 0.f) continue;
        const float2 g = reinterpret_cast<const float2*>(dU)[(size_t)img * H * W + (size_t)fy * W + fx];
        su += wy * wx * g.x;
        sv += wy * wx * g.y;
      }
    }
    float* d = dflow + i * 8;
    d[0] += 2.f * su;
    d[1] += 2.f * sv;
  }
}

// (dst blocks) += (src blocks), same geometry
__global__ void add_blocks_kernel(float* __restrict__ dst, int cbt_d, int cb_d,
                                  const float* __restrict__ src, int cbt_s, int cb_s, int nb,
                                  int n, int P) {
  const size_t total = (size_t)n * nb * P * 2;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int half = (int)(e & 1);
    const size_t r = e >> 1;
    const int p = (int)(r % P);
    const int b = (int)((r / P) % nb);
    const int img = (int)(r / ((size_t)P * nb));
    f4* d = reinterpret_cast<f4*>(dst + (((size_t)img * cbt_d + cb_d + b) * P + p) * 8) + half;
    *d += *(reinterpret_cast<const f4*>(src + (((size_t)img * cbt_s + cb_s + b) * P + p) * 8) + half);
  }
}

// ---------------------------------------------------------------- AdamW

__global__ void adamw_kernel(float* __restrict__ p, const float* __restrict__ g,
                             float* __restrict__ m, float* __restrict__ v, size_t n, float lr,
                             float b1, float b2, float eps, float wd, float bc1, float bc2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    float pi = p[i] * (1.f - lr * wd);
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    pi -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
  }
}

}  // namespace
}  // namespace tc

// ======================================================================
// trainer: buffers, the launch sequence and the C ABI

using namespace tc;

namespace {

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

struct TLayer {
  int cout, cin, stride, kc, cin_pad, np;  // forward geometry (packed input order)
  size_t woff, boff;                       // in the blob
  int* cmap;                               // device, cin_pad entries
  float *w, *b;                            // device, packed forward weights and bias
  float* wd;                               // device, packed data-gradient weights (stride 1)
  float* wu4 = nullptr;                    // device, F(4x4) Winograd forward weights, or null
  float* wud4 = nullptr;                   // device, F(4x4) Winograd data-gradient weights, or null
  int dcin, dnp;                           // data-gradient conv: input channels (pad 8), np
};

struct Level {
  int h, w, C;
  float *tmp, *feat;                // 2n images
  float *Z, *H1, *H23, *U, *flow;   // n images
  float *dflow, *dfeat;
};

}  // namespace

struct tc_trainer {
  tc_net_desc d;
  tc_train_params prm;
  int max_n, h, w, hp, wp, L, zcb, ncv;
  size_t nfl;
  int step;
  float *P, *G, *M, *V;  // blob layout
  TLayer pyr[8][2], dec[8][4];
  float* stage;
  Level lv[9];
  float *dH23, *dH1, *dZ, *T32, *W2, *dW2, *dU, *dTmp;
  float *cpart, *wpart, *bpart, *lpart, *loss, *zbias;
  size_t cpart_b, wpart_b;
  int lchunks;
  std::vector<void*> allocs;
};

namespace {

int tconv(const tc_trainer* t, const float* w, const float* b, int cout, int np, int nchunks,
          int kc, const View& in0, int nb0, const View& in1, int in_h, int in_w, float* out,
          int out_cbt, int out_cb0, int compact, const float* add, int out_h, int out_w, int relu,
          int n, int stride, hipStream_t s, const float* wu4 = nullptr) {
  ConvArgs a;
  memset(&a, 0, sizeof(a));
  a.in0 = in0;
  a.in1 = in1;
  a.nb0 = nb0;
  a.in_h = in_h;
  a.in_w = in_w;
  a.out = out;
  a.out_cbt = out_cbt;
  a.out_cb0 = out_cb0;
  a.compact = compact;
  a.add = add;
  a.out_h = out_h;
  a.out_w = out_w;
  a.w = w;
  a.b = b;
  a.nchunks = nchunks;
  a.nblk = nchunks * kc / 8;
  a.cout = cout;
  a.np = np;
  a.lrelu = relu;
  a.slope = t->d.leaky;
  a.n = n;
  a.partial = t->cpart;
  hipError_t e;
  if (wu4 && stride == 1 && kc == 8) {
    // F(4x4) Winograd weights packed for C_out rounded up to 32
    a.np = (cout + 31) / 32 * 32;
    a.splits = 1;
    a.cps = nchunks;
    e = launch_conv3x3_wino4(a, wu4, s);
  } else if (cout == 2 && compact && stride == 1 && kc == 8) {
    a.splits = 1;
    a.cps = nchunks;
    e = launch_head(a, s);
  } else {
    const ConvPlan p = plan_conv(out_h, out_w, n, nchunks, stride, np);
    if (conv_partial_bytes(p, out_h, out_w, n, np) > t->cpart_b) return TC_ERR_WORKSPACE;
    a.splits = p.splits;
    a.cps = p.cps;
    e = launch_conv3x3(a, stride, kc, p.mr, s);
  }
  return e == hipSuccess ? TC_OK : TC_ERR_HIP;
}

View view(const float* p, int cbt, int cb0 = 0) {
  View v;
  v.a = p;
  v.b = p;
  v.nsplit = 1 << 30;
  v.cbt = cbt;
  v.cb0 = cb0;
  v.tab = nullptr;
  return v;
}

// weight gradient of one layer: dz (blocked, dz_cbt blocks per image from
// dz_cb0), the forward input as up to two views; writes the gradient of W
// and b into the blob-layout gradient
int wgrad(tc_trainer* t, const TLayer& Ly, const float* dz, int dz_cbt, int dz_cb0,
          const float* x0, int x0_cbt, int x0_cb0, int nb0, const float* x1, int x1_cbt,
          int x1_cb0, int n, int ho, int wo, int hi, int wi, hipStream_t s) {
  WgArgs a;
  a.dz = dz;
  a.dz_cbt = dz_cbt;
  a.dz_cb0 = dz_cb0;
  a.x0 = x0;
  a.x0_cbt = x0_cbt;
  a.x0_cb0 = x0_cb0;
  a.nb0 = nb0;
  a.x1 = x1 ? x1 : x0;
  a.x1_cbt = x1_cbt;
  a.x1_cb0 = x1_cb0;
  a.n = n;
  a.ho = ho;
  a.wo = wo;
  a.hi = hi;
  a.wi = wi;
  a.stride = Ly.stride;
  const int KB = Ly.kc;
  a.nob = (Ly.cout + 7) / 8;
  a.ncb = Ly.cin_pad / KB;
  const long tiles = (long)n * ho * ((wo + WG_TW - 1) / WG_TW);
  const size_t chunk_b = (size_t)a.nob * a.ncb * 8 * KB * 9 * sizeof(float);
  // matrix cores: groups of up to 3 output blocks of 16 and of 16 input
  // channels; about 1024 workgroups over the pixel chunks
  const int mbt = (Ly.cout + 15) / 16, mb = std::min(mbt, 3), nmg = (mbt + mb - 1) / mb;
  const int ngrp = (Ly.cin_pad + 15) / 16;
  long chunks = 1024 / (ngrp * nmg);
  chunks = std::max(1L, std::min({chunks, tiles, (long)(t->wpart_b / chunk_b)}));
  a.chunks = (int)chunks;
  a.partial = t->wpart;
  dim3 grid(a.chunks, ngrp, nmg);
  const bool s1 = Ly.stride == 1;
  if (mb == 1)
    s1 ? wgrad_mfma_kernel<1, 1><<<grid, 256, 0, s>>>(a, KB, Ly.cout, Ly.cin_pad)
       : wgrad_mfma_kernel<1, 2><<<grid, 256, 0, s>>>(a, KB, Ly.cout, Ly.cin_pad);
  else if (mb == 2)
    s1 ? wgrad_mfma_kernel<2, 1><<<grid, 256, 0, s>>>(a, KB, Ly.cout, Ly.cin_pad)
       : wgrad_mfma_kernel<2, 2><<<grid, 256, 0, s>>>(a, KB, Ly.cout, Ly.cin_pad);
  else
    s1 ? wgrad_mfma_kernel<3, 1><<<grid, 256, 0, s>>>(a, KB, Ly.cout, Ly.cin_pad)
       : wgrad_mfma_kernel<3, 2><<<grid, 256, 0, s>>>(a, KB, Ly.cout, Ly.cin_pad);
  if (hipGetLastError() != hipSuccess) return TC_ERR_HIP;
  const int per_chunk = a.nob * a.ncb * 8 * KB * 9;
  wgrad_reduce_kernel<<<(per_chunk + 63) / 64, 256, 0, s>>>(t->wpart, a.chunks, a.nob, a.ncb, KB, Ly.cout,
                                                            Ly.cin, Ly.cin_pad, Ly.cmap, t->G, (int)Ly.woff);
  // bias
  const int bch = 256;
  bgrad_kernel<<<dim3(bch, a.nob), 256, 0, s>>>(dz, dz_cbt, dz_cb0, a.nob, n, ho * wo, bch,
                                                t->bpart);
  bgrad_reduce_kernel<<<Ly.cout, 256, 0, s>>>(t->bpart, bch, a.nob, Ly.cout, t->G, (int)Ly.boff);
  return hipGetLastError() == hipSuccess ? TC_OK : TC_ERR_HIP;
}

// data gradient of a stride-1 layer through the conv kernel
int dgrad(tc_trainer* t, const TLayer& Ly, const float* dz, int dz_cbt, int dz_cb0, float* out,
          int out_cbt, int out_cb0, int n, int h, int w, hipStream_t s) {
  return tconv(t, Ly.wd, t->zbias, Ly.cin_pad, Ly.dnp, Ly.dcin / 8, 8, view(dz, dz_cbt, dz_cb0),
               Ly.dcin / 8, view(dz, dz_cbt, dz_cb0), h, w, out, out_cbt, out_cb0, 0, nullptr, h,
               w, 0, n, 1, s, Ly.wud4);
}

#define TT(x)                      \
  do {                             \
    int st_ = (x);                 \
    if (st_) return st_;           \
  } while (0)
#define TH(x)                                  \
  do {                                         \
    if ((x) != hipSuccess) return TC_ERR_HIP;  \
  } while (0)

int pack_all(tc_trainer* t, hipStream_t s) {
  auto pk = [&](TLayer& Ly) {
    pack_fwd_kernel<<<grid1((size_t)Ly.cin_pad * 9 * Ly.np), 256, 0, s>>>(
        t->P, (int)Ly.woff, (int)Ly.boff, Ly.cout, Ly.cin, Ly.kc, Ly.cin_pad, Ly.np, Ly.cmap, Ly.w,
        Ly.b);
    if (Ly.wd)
      pack_dgrad_kernel<<<grid1((size_t)Ly.dcin * 9 * Ly.dnp), 256, 0, s>>>(
          t->P, (int)Ly.woff, Ly.cout, Ly.cin, Ly.dcin, Ly.dnp, Ly.cmap, Ly.cin_pad, Ly.wd);
    if (Ly.wu4) {
      const int nout = (Ly.cout + 31) / 32 * 32;
      pack_wino4_kernel<<<(nout * Ly.cin_pad + 255) / 256, 256, 0, s>>>(
          t->P, (int)Ly.woff, Ly.cout, Ly.cin, Ly.cmap, Ly.cin_pad, 0, nout, Ly.cin_pad, Ly.wu4);
    }
    if (Ly.wud4) {
      const int nout = (Ly.cin_pad + 31) / 32 * 32;
      pack_wino4_kernel<<<(nout * Ly.dcin + 255) / 256, 256, 0, s>>>(
          t->P, (int)Ly.woff, Ly.cout, Ly.cin, Ly.cmap, Ly.cin_pad, 1, nout, Ly.dcin, Ly.wud4);
    }
  };
  for (int l = 1; l <= t->L; ++l) {
    pk(t->pyr[l - 1][0]);
    pk(t->pyr[l - 1][1]);
    for (int k = 0; k < 4; ++k) pk(t->dec[l - 1][k]);
  }
  return hipGetLastError() == hipSuccess ? TC_OK : TC_ERR_HIP;
}

int forward(tc_trainer* t, const float* A, const float* B, int n, hipStream_t s) {
  const tc_net_desc& d = t->d;
  const int n2 = 2 * n;
  TH(launch_stage(A, n, t->h, t->w, t->stage, t->hp, t->wp, 0, nullptr, s));
  TH(launch_stage(B, n, t->h, t->w, t->stage + (size_t)n * t->hp * t->wp * 4, t->hp, t->wp, 0,
                  nullptr, s));
  const float* in = t->stage;
  int in_cbt = 1, ih = t->hp, iw = t->wp;
  for (int l = 1; l <= t->L; ++l) {
    Level& V = t->lv[l];
    const TLayer& La = t->pyr[l - 1][0];
    const TLayer& Lb = t->pyr[l - 1][1];
    TT(tconv(t, La.w, La.b, La.cout, La.np, La.cin_pad / La.kc, La.kc, view(in, in_cbt),
             La.cin_pad / La.kc, view(in, in_cbt), ih, iw, V.tmp, V.C / 8, 0, 0, nullptr, V.h,
             V.w, 1, n2, 2, s));
    TT(tconv(t, Lb.w, Lb.b, Lb.cout, Lb.np, Lb.cin_pad / 8, 8, view(V.tmp, V.C / 8), V.C / 8,
             view(V.tmp, V.C / 8), V.h, V.w, V.feat, V.C / 8, 0, 0, nullptr, V.h, V.w, 1, n2, 1, s));
    in = V.feat;
    in_cbt = V.C / 8;
    ih = V.h;
    iw = V.w;
  }
  const int d1b = d.dec[1] / 8, d23b = (d.dec[1] + d.dec[2]) / 8, d0b = d.dec[0] / 8;
  for (int l = t->L; l >= 1; --l) {
    Level& V = t->lv[l];
    const size_t fimg = (size_t)(V.C / 8) * V.h * V.w * 8;
    const float* Ul = nullptr;
    if (l < t->L) {
      TH(launch_up2x2(t->lv[l + 1].flow, n, t->lv[l + 1].h, t->lv[l + 1].w, V.U, s));
      Ul = V.U;
    }
    CvArgs cv;
    memset(&cv, 0, sizeof(cv));
    cv.f1 = view(V.feat, V.C / 8);
    cv.f2 = view(V.feat + n * fimg, V.C / 8);
    cv.U = Ul;
    cv.Z = V.Z;
    cv.zcb = t->zcb;
    cv.n = n;
    cv.h = V.h;
    cv.w = V.w;
    cv.C = V.C;
    cv.radius = d.radius;
    cv.slope = d.leaky;
    const CvPlan cp = plan_cost_volume(V.h, V.w, V.C);
    if (cost_volume_partial_bytes(cp, n, V.h, V.w) > t->cpart_b) return TC_ERR_WORKSPACE;
    cv.splits = cp.splits;
    cv.cps = cp.cps;
    cv.partial = t->cpart;
    TH(launch_warp_cost_volume(cv, s));
    const TLayer* Ld = t->dec[l - 1];
    TT(tconv(t, Ld[0].w, Ld[0].b, Ld[0].cout, Ld[0].np, Ld[0].cin_pad / 8, 8,
             view(V.feat, V.C / 8), V.C / 8, view(V.Z, t->zcb), V.h, V.w, V.H1, d0b, 0, 0, nullptr,
             V.h, V.w, 1, n, 1, s, Ld[0].wu4));
    TT(tconv(t, Ld[1].w, Ld[1].b, Ld[1].cout, Ld[1].np, Ld[1].cin_pad / 8, 8, view(V.H1, d0b),
             d0b, view(V.H1, d0b), V.h, V.w, V.H23, d23b, 0, 0, nullptr, V.h, V.w, 1, n, 1, s,
             Ld[1].wu4));
    TT(tconv(t, Ld[2].w, Ld[2].b, Ld[2].cout, Ld[2].np, Ld[2].cin_pad / 8, 8, view(V.H23, d23b),
             d1b, view(V.H23, d23b), V.h, V.w, V.H23, d23b, d1b, 0, nullptr, V.h, V.w, 1, n, 1, s,
             Ld[2].wu4));
    TT(tconv(t, Ld[3].w, Ld[3].b, 2, Ld[3].np, Ld[3].cin_pad / 8, 8, view(V.H23, d23b), d23b,
             view(V.H23, d23b), V.h, V.w, V.flow, 0, 0, 1, Ul, V.h, V.w, 0, n, 1, s));
  }
  return TC_OK;
}

int backward(tc_trainer* t, const float* T, int n, hipStream_t s) {
  const tc_net_desc& d = t->d;
  const int n2 = 2 * n;
  const float slope = d.leaky;
  const int d0b = d.dec[0] / 8, d1b = d.dec[1] / 8, d23b = (d.dec[1] + d.dec[2]) / 8;
  const int d2b = d.dec[2] / 8;
  TH(hipGetLastError());
  zero_kernel<<<grid1(t->nfl), 256, 0, s>>>(t->G, t->nfl);
  // loss and its gradient at every level
  int np_loss = 0;
  for (int l = 1; l <= t->L; ++l) {
    Level& V = t->lv[l];
    const float scale = 1.f / ((float)n * V.h * V.w);
    loss_kernel<<<t->lchunks, 256, 0, s>>>(V.flow, T, n, t->h, t->w, V.h, V.w, 1 << l,
                                          t->prm.loss_eps, t->prm.loss_q, scale, V.dflow,
                                          t->lpart + np_loss);
    np_loss += t->lchunks;
    zero_kernel<<<grid1((size_t)n2 * V.C * V.h * V.w), 256, 0, s>>>(
        V.dfeat, (size_t)n2 * V.C * V.h * V.w);
  }
  sum_kernel<<<1, 256, 0, s>>>(t->lpart, np_loss, t->loss);
  TH(hipGetLastError());

  for (int l = 1; l <= t->L; ++l) {
    Level& V = t->lv[l];
    const int h = V.h, w = V.w, P = h * w, C = V.C, cb = C / 8;
    const size_t fimg = (size_t)cb * P * 8;
    const TLayer* Ld = t->dec[l - 1];
    const int zt = cb + t->zcb;  // blocks of dZ: [F1 | CV | U | pad]
    // head: dflow (1 block) -> dH23; weight gradient from H23
    TT(wgrad(t, Ld[3], V.dflow, 1, 0, V.H23, d23b, 0, d23b, nullptr, 0, 0, n, h, w, h, w, s));
    TT(dgrad(t, Ld[3], V.dflow, 1, 0, t->dH23, d23b, 0, n, h, w, s));
    // c3: dz3 = dh3 * lrelu'(h3)
    lrelu_bwd_kernel<<<grid1((size_t)n * d2b * P * 2), 256, 0, s>>>(
        t->dH23, d23b, d1b, nullptr, 0, 0, V.H23, d23b, d1b, d2b, n, P, slope);
    TT(wgrad(t, Ld[2], t->dH23, d23b, d1b, V.H23, d23b, 0, d1b, nullptr, 0, 0, n, h, w, h, w, s));
    TT(dgrad(t, Ld[2], t->dH23, d23b, d1b, t->T32, d1b, 0, n, h, w, s));
    // c2: dz2 = (dh2 from the head + from c3) * lrelu'(h2)
    lrelu_bwd_kernel<<<grid1((size_t)n * d1b * P * 2), 256, 0, s>>>(
        t->dH23, d23b, 0, t->T32, d1b, 0, V.H23, d23b, 0, d1b, n, P, slope);
    TT(wgrad(t, Ld[1], t->dH23, d23b, 0, V.H1, d0b, 0, d0b, nullptr, 0, 0, n, h, w, h, w, s));
    TT(dgrad(t, Ld[1], t->dH23, d23b, 0, t->dH1, d0b, 0, n, h, w, s));
    // c1
    lrelu_bwd_kernel<<<grid1((size_t)n * d0b * P * 2), 256, 0, s>>>(
        t->dH1, d0b, 0, nullptr, 0, 0, V.H1, d0b, 0, d0b, n, P, slope);
    TT(wgrad(t, Ld[0], t->dH1, d0b, 0, V.feat, cb, 0, cb, V.Z, t->zcb, 0, n, h, w, h, w, s));
    TT(dgrad(t, Ld[0], t->dH1, d0b, 0, t->dZ, zt, 0, n, h, w, s));
    // cost volume -> F1 and the warped F2
    warp_kernel<<<grid1((size_t)n * P), 256, 0, s>>>(V.feat + n * fimg, l < t->L ? V.U : nullptr,
                                                     n, cb, h, w, t->W2);
    cv_bwd_f1_kernel<<<dim3((w + CV_T - 1) / CV_T, (h + CV_T - 1) / CV_T, n), 256, 0, s>>>(
        t->dZ, zt, cb, V.Z, t->zcb, slope, 1.f / C, t->W2, cb, n, h, w, V.dfeat);
    cv_bwd_f2w_kernel<<<dim3((w + CV_T - 1) / CV_T, (h + CV_T - 1) / CV_T, n), 256, 0, s>>>(
        t->dZ, zt, cb, V.Z, t->zcb, slope, 1.f / C, V.feat, cb, n, h, w, t->dW2);
    // warp backward; U = 2 up2(flow_{l+1}) below the top level
    const int ucb = cb + t->ncv / 8, uc = t->ncv % 8;
    warp_bwd_kernel<<<dim3((w + WB_T - 1) / WB_T, (h + WB_T - 1) / WB_T, n), 256, 0, s>>>(
        t->dW2, V.feat + n * fimg, l < t->L ? V.U : nullptr, n, cb, h, w, V.dfeat + n * fimg,
        t->dZ, zt, ucb, uc, V.dflow, l < t->L ? t->dU : nullptr);
    if (l < t->L) {
      Level& Vn = t->lv[l + 1];
      up2_bwd_kernel<<<grid1((size_t)n * Vn.h * Vn.w), 256, 0, s>>>(t->dU, n, Vn.h, Vn.w,
                                                                    Vn.dflow);
    }
    TH(hipGetLastError());
  }

  // pyramid, coarse to fine, both images of every pair
  for (int l = t->L; l >= 1; --l) {
    Level& V = t->lv[l];
    const int h = V.h, w = V.w, P = h * w, cb = V.C / 8;
    const TLayer& La = t->pyr[l - 1][0];
    const TLayer& Lb = t->pyr[l - 1][1];
    lrelu_bwd_kernel<<<grid1((size_t)n2 * cb * P * 2), 256, 0, s>>>(
        V.dfeat, cb, 0, nullptr, 0, 0, V.feat, cb, 0, cb, n2, P, slope);
    TT(wgrad(t, Lb, V.dfeat, cb, 0, V.tmp, cb, 0, cb, nullptr, 0, 0, n2, h, w, h, w, s));
    TT(dgrad(t, Lb, V.dfeat, cb, 0, t->dTmp, cb, 0, n2, h, w, s));
    lrelu_bwd_kernel<<<grid1((size_t)n2 * cb * P * 2), 256, 0, s>>>(
        t->dTmp, cb, 0, nullptr, 0, 0, V.tmp, cb, 0, cb, n2, P, slope);
    if (l == 1) {
      TT(wgrad(t, La, t->dTmp, cb, 0, t->stage, 1, 0, 1, nullptr, 0, 0, n2, h, w, t->hp, t->wp,
               s));
    } else {
      Level& Vp = t->lv[l - 1];
      const int pcb = Vp.C / 8;
      TT(wgrad(t, La, t->dTmp, cb, 0, Vp.feat, pcb, 0, pcb, nullptr, 0, 0, n2, h, w, Vp.h, Vp.w,
               s));
      dgrad_s2_kernel<<<dim3(1024, pcb), 256, 0, s>>>(t->dTmp, cb, t->P, (int)La.woff, La.cout,
                                                      La.cin, Vp.dfeat, n2, Vp.h, Vp.w, h, w);
    }
    TH(hipGetLastError());
  }
  return TC_OK;
}

bool trainer_desc_ok(const tc_net_desc* d) {
  if (!d || d->levels < 1 || d->levels > 6 || d->finest != 1 || d->ref_layers != 0) return false;
  if (d->radius != 4 || !(d->leaky > 0.f && d->leaky <= 1.f)) return false;
  for (int l = 0; l < d->levels; ++l)
    if (d->ch[l] <= 0 || d->ch[l] % 8 || d->ch[l] > 128) return false;
  for (int i = 0; i < 3; ++i)
    if (d->dec[i] <= 0 || d->dec[i] % 16 || d->dec[i] > 128) return false;
  const int zc = (81 + 2 + 7) / 8 * 8;
  for (int l = 0; l < d->levels; ++l)
    if (d->ch[l] + zc > 128) return false;       // c1 data gradient: one MFMA tile row
  if (d->dec[1] + d->dec[2] > 128) return false;
  return true;
}

}  // namespace

extern "C" {

void tc_train_default_params(tc_train_params* p) {
  if (!p) return;
  p->lr = 1e-4f;
  p->beta1 = 0.9f;
  p->beta2 = 0.99f;
  p->eps = 1e-8f;
  p->weight_decay = 4e-4f;
  p->loss_eps = 0.01f;
  p->loss_q = 0.4f;
}

void tc_trainer_destroy(tc_trainer* t) {
  if (!t) return;
  for (void* p : t->allocs) (void)hipFree(p);
  delete t;
}

int tc_trainer_create(const tc_net_desc* desc, const float* host_weights, size_t n_floats,
                      const tc_train_params* prm, int max_n, int h, int w, tc_trainer** out) {
  if (!desc || !host_weights || !prm || !out) return TC_ERR_INVALID_ARG;
  if (max_n < 1 || max_n > 64 || h < 1 || w < 1 || h > 4096 || w > 4096) return TC_ERR_INVALID_ARG;
  if (!trainer_desc_ok(desc)) return TC_ERR_SHAPE;
  if (n_floats != tc_weight_floats(desc)) return TC_ERR_SHAPE;
  tc_trainer* t = new (std::nothrow) tc_trainer();
  if (!t) return TC_ERR_HIP;
  t->d = *desc;
  t->prm = *prm;
  t->max_n = max_n;
  t->h = h;
  t->w = w;
  t->L = desc->levels;
  const int m = 1 << t->L;
  t->hp = (h + m - 1) / m * m;
  t->wp = (w + m - 1) / m * m;
  t->ncv = 81;
  t->zcb = (81 + 2 + 7) / 8;
  t->nfl = n_floats;
  t->step = 0;
  auto alloc = [&](size_t bytes) -> float* {
    void* p = nullptr;
    if (hipMalloc(&p, al(bytes ? bytes : 4)) != hipSuccess) return nullptr;
    t->allocs.push_back(p);
    return static_cast<float*>(p);
  };
  bool ok = true;
  auto A = [&](size_t bytes) {
    float* p = alloc(bytes);
    ok = ok && p;
    return p;
  };
  t->P = A(n_floats * 4);
  t->G = A(n_floats * 4);
  t->M = A(n_floats * 4);
  t->V = A(n_floats * 4);
  // layers in blob order
  size_t pos = 0;
  std::vector<std::pair<int*, std::vector<int>>> cmaps;
  auto layer = [&](TLayer& Ly, int cout, int cin, int stride, int kc, int cin_pad,
                   const std::vector<int>& cmap, bool data_grad) {
    Ly.cout = cout;
    Ly.cin = cin;
    Ly.stride = stride;
    Ly.kc = kc;
    Ly.cin_pad = cin_pad;
    Ly.np = (cout + 15) / 16 * 16;
    Ly.woff = pos;
    Ly.boff = pos + (size_t)cout * cin * 9;
    pos = Ly.boff + cout;
    Ly.cmap = reinterpret_cast<int*>(A(cin_pad * sizeof(int)));
    cmaps.push_back({Ly.cmap, cmap});
    Ly.w = A((size_t)cin_pad * 9 * Ly.np * 4);
    Ly.b = A((size_t)Ly.np * 4);
    Ly.dcin = (cout + 7) / 8 * 8;
    Ly.dnp = (cin_pad + 15) / 16 * 16;
    Ly.wd = data_grad ? A((size_t)Ly.dcin * 9 * Ly.dnp * 4) : nullptr;
  };
  auto ident = [](int cin, int pad) {
    std::vector<int> v(pad, -1);
    for (int c = 0; c < cin; ++c) v[c] = c;
    return v;
  };
  for (int l = 1; l <= t->L; ++l) {
    const int C = desc->ch[l - 1], cin = l == 1 ? 3 : desc->ch[l - 2];
    const int kc = l == 1 ? 4 : 8, pad = l == 1 ? 4 : cin;
    layer(t->pyr[l - 1][0], C, cin, 2, kc, pad, ident(cin, pad), false);
    layer(t->pyr[l - 1][1], C, C, 1, 8, C, ident(C, C), true);
  }
  const int d0 = desc->dec[0], d1 = desc->dec[1], d2 = desc->dec[2];
  for (int l = 1; l <= t->L; ++l) {
    const int C = desc->ch[l - 1];
    const int pad = C + t->zcb * 8;
    std::vector<int> mp(pad, -1);  // packed [F1 | CV | U | pad] <- blob [CV | F1 | U]
    for (int g = 0; g < C; ++g) mp[g] = 81 + g;
    for (int k = 0; k < 81; ++k) mp[C + k] = k;
    mp[C + 81] = 81 + C;
    mp[C + 82] = 81 + C + 1;
    layer(t->dec[l - 1][0], d0, 81 + C + 2, 1, 8, pad, mp, true);
    layer(t->dec[l - 1][1], d1, d0, 1, 8, d0, ident(d0, d0), true);
    layer(t->dec[l - 1][2], d2, d1, 1, 8, d1, ident(d1, d1), true);
    layer(t->dec[l - 1][3], 2, d1 + d2, 1, 8, d1 + d2, ident(d1 + d2, d1 + d2), true);
  }
  if (pos != n_floats) ok = false;
  // activations
  const int n = max_n, n2 = 2 * n;
  t->stage = A((size_t)n2 * t->hp * t->wp * 16);
  size_t maxP = 0;
  for (int l = 1; l <= t->L; ++l) {
    Level& V = t->lv[l];
    V.h = t->hp >> l;
    V.w = t->wp >> l;
    V.C = desc->ch[l - 1];
    const size_t P = (size_t)V.h * V.w;
    maxP = std::max(maxP, P);
    V.tmp = A((size_t)n2 * V.C * P * 4);
    V.feat = A((size_t)n2 * V.C * P * 4);
    V.Z = A((size_t)n * t->zcb * 8 * P * 4);
    V.H1 = A((size_t)n * d0 * P * 4);
    V.H23 = A((size_t)n * (d1 + d2) * P * 4);
    V.U = A((size_t)n * 2 * P * 4);
    V.flow = A((size_t)n * 2 * P * 4);
    V.dflow = A((size_t)n * 8 * P * 4);
    V.dfeat = A((size_t)n2 * V.C * P * 4);
  }
  // F(4x4) Winograd for the decoder convs of levels with at least 128
  // regions of 16 x 32 output pixels per image, where rounding the conv's
  // outputs up to 32 adds at most a third (c1 and c2 forward; c1, c2 and c3
  // data gradient at the student's sizes)
  for (int l = 1; l <= t->L; ++l) {
    const Level& V = t->lv[l];
    if ((long)((V.w + 31) / 32) * ((V.h + 15) / 16) < 128) continue;
    auto fits = [](int nout) { return 3 * ((nout + 31) / 32 * 32) <= 4 * nout; };
    for (int k = 0; k < 3; ++k) {
      TLayer& Ly = t->dec[l - 1][k];
      if (fits(Ly.cout)) Ly.wu4 = A((size_t)(Ly.cout + 31) / 32 * 32 * Ly.cin_pad * 36 * 4);
      if (Ly.wd && fits(Ly.cin_pad)) Ly.wud4 = A((size_t)(Ly.cin_pad + 31) / 32 * 32 * Ly.dcin * 36 * 4);
    }
  }
  int maxC = 0;
  for (int l = 0; l < t->L; ++l) maxC = std::max(maxC, desc->ch[l]);
  t->dH23 = A((size_t)n * (d1 + d2) * maxP * 4);
  t->dH1 = A((size_t)n * d0 * maxP * 4);
  t->dZ = A((size_t)n * (maxC + t->zcb * 8) * maxP * 4);
  t->T32 = A((size_t)n * d1 * maxP * 4);
  t->W2 = A((size_t)n * maxC * maxP * 4);
  t->dW2 = A((size_t)n * maxC * maxP * 4);
  t->dU = A((size_t)n * 2 * maxP * 4);
  t->dTmp = A((size_t)n2 * maxC * maxP * 4);
  // split-K partials of the convs (forward and data gradient) and the cost volume
  size_t cp = 0;
  for (int l = 1; l <= t->L; ++l) {
    const Level& V = t->lv[l];
    for (int k = 0; k < 2; ++k) {
      const TLayer& Ly = t->pyr[l - 1][k];
      cp = std::max(cp, conv_partial_bytes(plan_conv(V.h, V.w, n2, Ly.cin_pad / Ly.kc, Ly.stride,
                                                     Ly.np), V.h, V.w, n2, Ly.np));
      if (Ly.wd)
        cp = std::max(cp, conv_partial_bytes(plan_conv(V.h, V.w, n2, Ly.dcin / 8, 1, Ly.dnp), V.h,
                                             V.w, n2, Ly.dnp));
    }
    for (int k = 0; k < 4; ++k) {
      const TLayer& Ly = t->dec[l - 1][k];
      cp = std::max(cp, conv_partial_bytes(plan_conv(V.h, V.w, n, Ly.cin_pad / 8, 1, Ly.np), V.h,
                                           V.w, n, Ly.np));
      cp = std::max(cp, conv_partial_bytes(plan_conv(V.h, V.w, n, Ly.dcin / 8, 1, Ly.dnp), V.h,
                                           V.w, n, Ly.dnp));
    }
    cp = std::max(cp, cost_volume_partial_bytes(plan_cost_volume(V.h, V.w, V.C), n, V.h, V.w));
  }
  t->cpart_b = cp;
  t->cpart = A(cp);
  t->wpart_b = (size_t)32 << 20;
  t->wpart = A(t->wpart_b);
  t->bpart = A((size_t)256 * 16 * 8 * 4);
  t->lchunks = 256;
  t->lpart = A((size_t)t->lchunks * t->L * 4);
  t->loss = A(16);
  t->zbias = A(256 * 4);
  if (!ok) {
    tc_trainer_destroy(t);
    return TC_ERR_HIP;
  }
  for (auto& cm : cmaps)
    if (hipMemcpy(cm.first, cm.second.data(), cm.second.size() * sizeof(int),
                  hipMemcpyHostToDevice) != hipSuccess)
      ok = false;
  if (ok && hipMemcpy(t->P, host_weights, n_floats * 4, hipMemcpyHostToDevice) != hipSuccess) ok = false;
  if (ok && (hipMemset(t->M, 0, n_floats * 4) != hipSuccess ||
             hipMemset(t->V, 0, n_floats * 4) != hipSuccess ||
             hipMemset(t->zbias, 0, 256 * 4) != hipSuccess))
    ok = false;
  if (ok && hipDeviceSynchronize() != hipSuccess) ok = false;
  if (!ok) {
    tc_trainer_destroy(t);
    return TC_ERR_HIP;
  }
  *out = t;
  return TC_OK;
}

int tc_trainer_grad(tc_trainer* t, const float* A, const float* B, const float* teacher, int n,
                    float* loss_out, hipStream_t stream) {
  if (!t || !A || !B || !teacher || n < 1 || n > t->max_n) return TC_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  int st = pack_all(t, s);
  if (st) return st;
  st = forward(t, A, B, n, s);
  if (st) return st;
  st = backward(t, teacher, n, s);
  if (st) return st;
  if (loss_out && hipMemcpyAsync(loss_out, t->loss, 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return TC_ERR_HIP;
  return TC_OK;
}

int tc_trainer_step(tc_trainer* t, const float* A, const float* B, const float* teacher, int n,
                    float* loss_out, hipStream_t stream) {
  int st = tc_trainer_grad(t, A, B, teacher, n, loss_out, stream);
  if (st) return st;
  t->step += 1;
  const double bc1 = 1.0 - pow((double)t->prm.beta1, t->step);
  const double bc2 = 1.0 - pow((double)t->prm.beta2, t->step);
  adamw_kernel<<<grid1(t->nfl), 256, 0, (hipStream_t)stream>>>(
      t->P, t->G, t->M, t->V, t->nfl, t->prm.lr, t->prm.beta1, t->prm.beta2, t->prm.eps,
      t->prm.weight_decay, (float)bc1, (float)bc2);
  return hipGetLastError() == hipSuccess ? TC_OK : TC_ERR_HIP;
}

int tc_trainer_copy(const tc_trainer* t, int which, float* dst, hipStream_t stream) {
  if (!t || !dst || which < 0 || which > 3) return TC_ERR_INVALID_ARG;
  const float* src = which == 0 ? t->P : which == 1 ? t->G : which == 2 ? t->M : t->V;
  return hipMemcpyAsync(dst, src, t->nfl * 4, hipMemcpyDefault, (hipStream_t)stream) == hipSuccess
             ? TC_OK
             : TC_ERR_HIP;
}

int tc_trainer_steps_done(const tc_trainer* t) { return t ? t->step : -1; }

}  // extern "C"
