// Depthwise separable layer of the refinement network (Sec. 3.2, "-sepref"):
// a dilated depthwise 3x3 conv followed by a pointwise conv, fused.
//
// The pointwise conv is a GEMM (M = pixels, N = output channels, K = input
// channels) on the matrix cores; its A operand is the depthwise output, which
// every lane computes itself for the pixel and channels it supplies to the
// MFMA (9 dilated taps read from global memory / cache, FP32 arithmetic), so
// the depthwise result never goes to memory.  A wave owns MR blocks of 16
// consecutive pixels of one image and all output channels; a lane's
// pointwise weights for the next K chunk are fetched while the current chunk
// runs.
//
// FP32 form, v_mfma_f32_16x16x4_f32 with K chunks of 16 channels: lane group
// g = l / 16 holds channels 4g .. 4g+3 of the chunk for pixel l % 16 and
// feeds them to four MFMAs, one channel each (the weights are packed in the
// same order).  BF16 form, v_mfma_f32_16x16x32_bf16 with K chunks of 32
// channels: lane group g holds channels 8g .. 8g+7.  Accumulation is FP32 in
// both; D[m = 4 (l / 16) + v][n = l % 16].
#include <type_traits>

#include "act.h"
#include "tc_internal.h"

namespace tc {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kSepMR = 2;  // 16-pixel blocks per wave

template <bool BF>
struct SepTraits {
  using T = float;                  // stored activation type
  using Frag = f4;                  // a lane's pointwise weights of one chunk
  static constexpr int CH = 4;      // channels a lane supplies per chunk
};
template <>
struct SepTraits<true> {
  using T = bf16;
  using Frag = u4;
  static constexpr int CH = 8;
};

// CH channels of input block `blk` (sub-block `part` of CH channels) at one
// pixel, zero where the block does not exist.
template <bool BF>
__device__ inline void load_in(const SepArgs& a, int img, int blk, int part, size_t pix,
                               float (&v)[SepTraits<BF>::CH]) {
  constexpr int CH = SepTraits<BF>::CH;
  if (blk < a.nblk) {
    const size_t plane = (size_t)a.h * a.w;
    if constexpr (BF) {
      const bf16* p = reinterpret_cast<const bf16*>(a.in) +
                      (((size_t)img * a.in_cbt + blk) * plane + pix) * 8;
      load8(p, v);
    } else {
      const float* p = reinterpret_cast<const float*>(a.in) +
                       (((size_t)img * a.in_cbt + blk) * plane + pix) * 8 + part * 4;
      const f4 x = *reinterpret_cast<const f4*>(p);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < CH; ++i) v[i] = 0.f;
  if (blk == a.nblk && a.flow && part == 0) {
    const float2 f = reinterpret_cast<const float2*>(a.flow)[(size_t)img * a.h * a.w + pix];
    v[0] = f.x;
    v[1] = f.y;
  }
}

template <bool BF, int NB>
__global__ __launch_bounds__(256) void sepconv_mfma(SepLayer L, SepArgs a) {
  using Tr = SepTraits<BF>;
  using Frag = typename Tr::Frag;
  constexpr int CH = Tr::CH;
  constexpr int K = 4 * CH;  // channels per chunk
  constexpr int MR = kSepMR;
  __shared__ f4 s_dw[9 * kSepMaxC / 4];
  __shared__ f4 s_dwb[kSepMaxC / 4];

  const int cin_pad = L.cin_pad;
  for (int i = threadIdx.x; i < 9 * cin_pad / 4; i += blockDim.x)
    s_dw[i] = reinterpret_cast<const f4*>(L.dw)[i];
  for (int i = threadIdx.x; i < cin_pad / 4; i += blockDim.x)
    s_dwb[i] = reinterpret_cast<const f4*>(L.dwb)[i];
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lm = lane & 15, lg = lane >> 4;
  const int img = blockIdx.y;
  const int hw = a.h * a.w;
  const int p0 = (blockIdx.x * 4 + wave) * (16 * MR);
  if (p0 >= hw) return;  // no barrier follows

  int py[MR], px[MR];
  bool ok[MR];
#pragma unroll
  for (int mb = 0; mb < MR; ++mb) {
    const int p = p0 + mb * 16 + lm;
    ok[mb] = p < hw;
    py[mb] = ok[mb] ? p / a.w : 0;
    px[mb] = ok[mb] ? p - py[mb] * a.w : 0;
  }

  f4 acc[MR][NB];
#pragma unroll
  for (int mb = 0; mb < MR; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};

  const int nchunks = cin_pad / K;
  const Frag* wsrc = reinterpret_cast<const Frag*>(L.pw);
  Frag fb[NB], fbn[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) fb[nb] = wsrc[nb * 64 + lane];

  const int d = L.dil;
  for (int c = 0; c < nchunks; ++c) {
    if (c + 1 < nchunks) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) fbn[nb] = wsrc[((size_t)(c + 1) * NB + nb) * 64 + lane];
    }
    // this lane's channels: ch0 .. ch0 + CH - 1, in input block blk
    const int ch0 = c * K + lg * CH;
    const int blk = ch0 >> 3, part = (ch0 & 7) / CH;
#pragma unroll
    for (int mb = 0; mb < MR; ++mb) {
      float t[CH];
      {
        const f4* bb = s_dwb + ch0 / 4;
#pragma unroll
        for (int i = 0; i < CH / 4; ++i) {
          const f4 b4 = bb[i];
          t[4 * i] = b4.x; t[4 * i + 1] = b4.y; t[4 * i + 2] = b4.z; t[4 * i + 3] = b4.w;
        }
      }
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = py[mb] + (tap / 3 - 1) * d, xx = px[mb] + (tap % 3 - 1) * d;
        if (!ok[mb] || yy < 0 || yy >= a.h || xx < 0 || xx >= a.w) continue;
        float v[CH];
        load_in<BF>(a, img, blk, part, (size_t)yy * a.w + xx, v);
        const f4* wt = s_dw + (tap * cin_pad + ch0) / 4;
#pragma unroll
        for (int i = 0; i < CH / 4; ++i) {
          const f4 w4 = wt[i];
          t[4 * i] += w4.x * v[4 * i];
          t[4 * i + 1] += w4.y * v[4 * i + 1];
          t[4 * i + 2] += w4.z * v[4 * i + 2];
          t[4 * i + 3] += w4.w * v[4 * i + 3];
        }
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) t[i] = t[i] >= 0.f ? t[i] : a.slope * t[i];
      if constexpr (BF) {
        const u4 fa = u4{pack2(t[0], t[1]), pack2(t[2], t[3]), pack2(t[4], t[5]), pack2(t[6], t[7])};
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf8, fa), __builtin_bit_cast(bf8, fb[nb]), acc[mb][nb], 0, 0, 0);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(t[j], fb[nb][j], acc[mb][nb], 0, 0, 0);
      }
    }
    if (c + 1 < nchunks) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) fb[nb] = fbn[nb];
    }
  }

  // epilogue: lane holds pixels p0 + 16 mb + 4 lg + v, output channel 16 nb + lm
  const size_t plane = (size_t)hw;
#pragma unroll
  for (int mb = 0; mb < MR; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int o = nb * 16 + lm;
      if (o >= L.cout) continue;
      const float bo = L.b[o];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = p0 + mb * 16 + 4 * lg + v;
        if (p >= hw) continue;
        float r = acc[mb][nb][v] + bo;
        if (a.lrelu) r = r >= 0.f ? r : a.slope * r;
        if (a.add) {
          const size_t q = ((size_t)img * plane + p) * 2 + o;
          reinterpret_cast<float*>(a.out)[q] = a.add[q] + r;
        } else {
          store1(reinterpret_cast<typename Tr::T*>(a.out) +
                     (((size_t)img * a.out_cbt + (o >> 3)) * plane + p) * 8 + (o & 7),
                 r);
        }
      }
    }
}

template <bool BF>
hipError_t dispatch_sep(const SepLayer& L, const SepArgs& a, dim3 grid, hipStream_t s) {
  switch (L.np / 16) {
    case 1: sepconv_mfma<BF, 1><<<grid, 256, 0, s>>>(L, a); break;
    case 2: sepconv_mfma<BF, 2><<<grid, 256, 0, s>>>(L, a); break;
    case 3: sepconv_mfma<BF, 3><<<grid, 256, 0, s>>>(L, a); break;
    case 4: sepconv_mfma<BF, 4><<<grid, 256, 0, s>>>(L, a); break;
    case 5: sepconv_mfma<BF, 5><<<grid, 256, 0, s>>>(L, a); break;
    case 6: sepconv_mfma<BF, 6><<<grid, 256, 0, s>>>(L, a); break;
    case 7: sepconv_mfma<BF, 7><<<grid, 256, 0, s>>>(L, a); break;
    case 8: sepconv_mfma<BF, 8><<<grid, 256, 0, s>>>(L, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sepconv(const SepLayer& L, const SepArgs& a, hipStream_t s) {
  const int K = L.bf16 ? 32 : 16;
  if (L.cin_pad <= 0 || L.cin_pad % K || L.cin_pad > kSepMaxC) return hipErrorInvalidValue;
  if (8 * (a.nblk + (a.flow ? 1 : 0)) > L.cin_pad) return hipErrorInvalidValue;
  if (L.np % 16 || L.np < L.cout || (a.add && L.cout != 2)) return hipErrorInvalidValue;
  const long hw = (long)a.h * a.w;
  if (a.n <= 0 || hw <= 0) return hipSuccess;
  const long tiles = (hw + 16 * kSepMR - 1) / (16 * kSepMR);
  dim3 grid((unsigned)((tiles + 3) / 4), (unsigned)a.n);
  return L.bf16 ? dispatch_sep<true>(L, a, grid, s) : dispatch_sep<false>(L, a, grid, s);
}

}  // namespace tc
