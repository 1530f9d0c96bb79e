// 3x3 convolution (zero padding 1, stride 1 or 2) as an implicit GEMM on the
// FP32 matrix cores of gfx950 (v_mfma_f32_16x16x4_f32).
//
// GEMM view: M = output pixels, N = output channels, K = 9 taps x input
// channels.  A workgroup (4 waves) owns an 8 x 16 tile of output pixels and
// every output channel; wave w computes output rows 2w and 2w+1 of the tile
// (two 16-pixel M blocks) against NB 16-channel N blocks.  K runs over input
// channel chunks of KC (= the block size of the input layout): per chunk the
// input halo tile and the chunk's weights are staged in LDS, then 9 * KC / 4
// MFMA steps consume them.
//
// MFMA 16x16x4 f32 operand layout (lane l of 64):
//   A (16 x 4):  A[m = l % 16][k = l / 16]
//   B (4 x 16):  B[k = l / 16][n = l % 16]
//   D (16 x 16): D[m = 4 * (l / 16) + v][n = l % 16] in accumulator VGPR v.
#include "tc_internal.h"

namespace tc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TH = 8, TW = 16;

// LDS row pitch that puts the four 16-lane groups of an MFMA operand read on
// distinct bank ranges (pitch = 16 mod 32).
__host__ __device__ constexpr int pitch16(int n) { return (n % 32 == 16) ? n : (n / 32) * 32 + 48; }

__device__ inline const float* view_base(const View& v, int img, size_t img_floats) {
  return img < v.nsplit ? v.a + (size_t)img * img_floats
                        : v.b + (size_t)(img - v.nsplit) * img_floats;
}

template <int S, int KC, int NB>
__global__ __launch_bounds__(256) void conv3x3_f32_mfma(ConvArgs a) {
  constexpr int IH = (TH - 1) * S + 3, IW = (TW - 1) * S + 3;
  constexpr int NPOS = IH * IW;
  constexpr int APITCH = pitch16(NPOS);
  constexpr int NP = NB * 16;
  constexpr int BPITCH = pitch16(NP);
  __shared__ float sA[KC * APITCH];
  __shared__ float sB[9 * KC * BPITCH];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int tx0 = blockIdx.x * TW, ty0 = blockIdx.y * TH, img = blockIdx.z;
  const int iy0 = ty0 * S - 1, ix0 = tx0 * S - 1;
  const size_t in_plane = (size_t)a.in_h * a.in_w * KC;

  f4 acc[2][NB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const int lm = lane & 15, lk = lane >> 4;

  for (int ch = 0; ch < a.nchunks; ++ch) {
    // ---- stage the input halo tile of this channel chunk: sA[c][pos]
    const View& v = ch < a.nb0 ? a.in0 : a.in1;
    const int cb = (ch < a.nb0 ? ch : ch - a.nb0) + v.cb0;
    const float* src = view_base(v, img, in_plane * v.cbt) + (size_t)cb * in_plane;
    for (int i = tid; i < NPOS * (KC / 4); i += 256) {
      const int pos = i / (KC / 4), c4 = i % (KC / 4);
      const int py = pos / IW, px = pos - py * IW;
      const int gy = iy0 + py, gx = ix0 + px;
      f4 val = f4{0.f, 0.f, 0.f, 0.f};
      if (gy >= 0 && gy < a.in_h && gx >= 0 && gx < a.in_w)
        val = *reinterpret_cast<const f4*>(src + ((size_t)gy * a.in_w + gx) * KC + c4 * 4);
      sA[(c4 * 4 + 0) * APITCH + pos] = val.x;
      sA[(c4 * 4 + 1) * APITCH + pos] = val.y;
      sA[(c4 * 4 + 2) * APITCH + pos] = val.z;
      sA[(c4 * 4 + 3) * APITCH + pos] = val.w;
    }
    // ---- stage the chunk's weights: sB[tap * KC + c][n]
    const f4* wsrc = reinterpret_cast<const f4*>(a.w + (size_t)ch * 9 * KC * NP);
    for (int i = tid; i < 9 * KC * NP / 4; i += 256) {
      const int row = i / (NP / 4), col = (i % (NP / 4)) * 4;
      const f4 val = wsrc[i];
      float* d = sB + row * BPITCH + col;
      d[0] = val.x;
      d[1] = val.y;
      d[2] = val.z;
      d[3] = val.w;
    }
    __syncthreads();

#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int p = tap / 3, q = tap % 3;
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
        float bf[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bf[nb] = sB[(tap * KC + kk * 4 + lk) * BPITCH + nb * 16 + lm];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          const int r = wave * 2 + mb;
          const float af = sA[(kk * 4 + lk) * APITCH + (r * S + p) * IW + lm * S + q];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf[nb], acc[mb][nb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // ---- epilogue: bias, LeakyReLU, optional flow accumulation, store
  const size_t out_plane = (size_t)a.out_h * a.out_w * 8;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    const int oy = ty0 + wave * 2 + mb;
    if (oy >= a.out_h) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int n = nb * 16 + lm;
      if (n >= a.cout) continue;
      const float bias = a.b[n];
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int ox = tx0 + 4 * lk + vv;
        if (ox >= a.out_w) continue;
        float val = acc[mb][nb][vv] + bias;
        if (a.lrelu) val = val >= 0.f ? val : a.slope * val;
        const size_t pix = ((size_t)img * a.out_h + oy) * a.out_w + ox;
        if (a.compact) {
          if (a.add) val += a.add[pix * a.cout + n];
          a.out[pix * a.cout + n] = val;
        } else {
          float* dst = a.out + (size_t)img * a.out_cbt * out_plane +
                       (size_t)(a.out_cb0 + (n >> 3)) * out_plane +
                       ((size_t)oy * a.out_w + ox) * 8 + (n & 7);
          *dst = val;
        }
      }
    }
  }
}

template <int S, int KC>
hipError_t dispatch_nb(const ConvArgs& a, hipStream_t s) {
  dim3 grid(cdiv(a.out_w, TW), cdiv(a.out_h, TH), a.n);
  switch (a.np / 16) {
    case 1: conv3x3_f32_mfma<S, KC, 1><<<grid, 256, 0, s>>>(a); break;
    case 2: conv3x3_f32_mfma<S, KC, 2><<<grid, 256, 0, s>>>(a); break;
    case 3: conv3x3_f32_mfma<S, KC, 3><<<grid, 256, 0, s>>>(a); break;
    case 4: conv3x3_f32_mfma<S, KC, 4><<<grid, 256, 0, s>>>(a); break;
    case 5: conv3x3_f32_mfma<S, KC, 5><<<grid, 256, 0, s>>>(a); break;
    case 6: conv3x3_f32_mfma<S, KC, 6><<<grid, 256, 0, s>>>(a); break;
    case 7: conv3x3_f32_mfma<S, KC, 7><<<grid, 256, 0, s>>>(a); break;
    case 8: conv3x3_f32_mfma<S, KC, 8><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_conv3x3(const ConvArgs& a, int stride, int kc, hipStream_t s) {
  if (a.n <= 0 || a.out_h <= 0 || a.out_w <= 0) return hipSuccess;
  if (stride == 1 && kc == 8) return dispatch_nb<1, 8>(a, s);
  if (stride == 2 && kc == 8) return dispatch_nb<2, 8>(a, s);
  if (stride == 2 && kc == 4) return dispatch_nb<2, 4>(a, s);
  if (stride == 1 && kc == 4) return dispatch_nb<1, 4>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace tc
