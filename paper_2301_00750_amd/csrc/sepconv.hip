// Depthwise separable layer of the refinement network (Sec. 3.2, "-sepref"):
// a dilated depthwise 3x3 conv followed by a pointwise conv, fused.
//
// The pointwise conv is a GEMM (M = pixels, N = output channels, K = input
// channels) on the matrix cores; its A operand is the depthwise output, which
// every lane computes itself for the pixel and channels it supplies to the
// MFMA (9 dilated taps read from global memory / cache, FP32 arithmetic), so
// the depthwise result never goes to memory.  A wave owns 16 consecutive
// pixels of one image and all output channels; the layer's weights sit in
// LDS, and the taps of the next K chunk load while the current chunk
// computes.  Workgroups are persistent over a contiguous range of tiles.
//
// Depthwise arithmetic: FP32 FMAs in the FP32 form; in the BF16 form
// v_dot2_f32_bf16 over pairs of taps with bfloat16 weights (FP32 sums).
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

template <bool BF>
struct SepTraits {
  using T = float;                  // stored activation type
  using Frag = f4;                  // a lane's pointwise weights of one chunk
  using Raw = f4;                   // a lane's input of one tap as stored
  static constexpr int CH = 4;      // channels a lane supplies per chunk
};
template <>
struct SepTraits<true> {
  using T = bf16;
  using Frag = u4;
  using Raw = u4;
  static constexpr int CH = 8;
};

// One tap of a lane's input as stored: CH channels (4 floats, or 8 bfloat16)
// of one pixel, from the chunk's channel block.
template <bool BF>
__device__ inline typename SepTraits<BF>::Raw load_raw(const typename SepTraits<BF>::T* base,
                                                       int pix) {
  return *reinterpret_cast<const typename SepTraits<BF>::Raw*>(base + (size_t)pix * 8);
}

template <bool BF>
__device__ inline void unpack_raw(const typename SepTraits<BF>::Raw& r,
                                  float (&v)[SepTraits<BF>::CH]) {
  if constexpr (BF) {
    load8(reinterpret_cast<const bf16*>(&r), v);
  } else {
    v[0] = r.x; v[1] = r.y; v[2] = r.z; v[3] = r.w;
  }
}

// LDS copy of n 16-byte words with 8 loads in flight per thread.
template <typename W>
__device__ inline void stage_lds(W* dst, const W* src, int n) {
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * blockDim.x) {
    W r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = i0 + k * blockDim.x;
      r[k] = i < n ? src[i] : W{};
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = i0 + k * blockDim.x;
      if (i < n) dst[i] = r[k];
    }
  }
}

template <bool BF, int NB>
__global__ __launch_bounds__(256, 2) void sepconv_mfma(SepLayer L, SepArgs a) {
  using Tr = SepTraits<BF>;
  using T = typename Tr::T;
  using Frag = typename Tr::Frag;
  using Raw = typename Tr::Raw;
  constexpr int CH = Tr::CH;
  constexpr int K = 4 * CH;  // channels per chunk
  __shared__ Frag s_pw[kSepPwFloats * 4 / sizeof(Frag)];
  __shared__ f4 s_dw[9 * kSepMaxC / 4];
  __shared__ f4 s_dwb[kSepMaxC / 4];

  // weights of the layer into LDS, once per workgroup
  const int cin_pad = L.cin_pad;
  const int nchunks = cin_pad / K;
  stage_lds(s_pw, reinterpret_cast<const Frag*>(L.pw), nchunks * NB * 64);
  if constexpr (BF)  // depthwise weights as bfloat16 pairs of taps (2p, 2p+1), p < 5
    stage_lds(reinterpret_cast<u4*>(s_dw), reinterpret_cast<const u4*>(L.dw2), 5 * cin_pad / 4);
  else
    stage_lds(s_dw, reinterpret_cast<const f4*>(L.dw), 9 * cin_pad / 4);
  stage_lds(s_dwb, reinterpret_cast<const f4*>(L.dwb), cin_pad / 4);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lm = lane & 15, lg = lane >> 4;
  const int hw = a.h * a.w;
  const int tpi = (hw + 15) / 16;  // wave tiles (16 pixels) per image
  const int total = a.n * tpi;
  // each workgroup takes a contiguous range of wave tiles; the workgroups of
  // one XCD (round-robin dispatch) take neighbouring ranges, so the dilated
  // taps of a region are served by one L2
  const int G = gridDim.x;
  const int wg = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const int per = (total + G - 1) / G;
  const int t_end = min(total, (wg + 1) * per);
  const int d = L.dil;
  const size_t plane = (size_t)hw;

  for (int wt = wg * per + wave; wt < t_end; wt += 4) {
    const int img = wt / tpi;
    const int p0 = (wt - img * tpi) * 16;
    // input pixel of every tap, -1 outside the image (zero padding)
    int off[9];
    bool all_in = true;
    {
      const int p = p0 + lm;
      const int y = p / a.w, x = p - (p / a.w) * a.w;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + (tap / 3 - 1) * d, xx = x + (tap % 3 - 1) * d;
        const bool in = p < hw && yy >= 0 && yy < a.h && xx >= 0 && xx < a.w;
        off[tap] = in ? yy * a.w + xx : -1;
        all_in = all_in && in;
      }
    }
    // wave-uniform: no tap of this tile leaves the image
    const bool interior = __all(all_in);

    f4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};

    // Taps of a chunk as stored.  Loads are unconditional (clamped to the
    // image and to the last stored block: padded channels have zero
    // weights); out-of-image taps are zeroed when used.
    auto fetch = [&](Raw (&raw)[9], int c) {
      const int ch0 = c * K + lg * CH;
      const int blk = min(ch0 >> 3, a.nblk - 1), part = (ch0 & 7) / CH;
      const T* base = reinterpret_cast<const T*>(a.in) +
                      ((size_t)img * a.in_cbt + blk) * plane * 8 + part * CH;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) raw[tap] = load_raw<BF>(base, max(off[tap], 0));
    };
    // depthwise taps + bias + LeakyReLU -> A operand, then the chunk's MFMAs
    auto compute = [&](const Raw (&raw)[9], int c) {
      const int ch0 = c * K + lg * CH;
      float t[CH];
#pragma unroll
      for (int i = 0; i < CH / 4; ++i) {
        const f4 b4 = s_dwb[ch0 / 4 + i];
        t[4 * i] = b4.x; t[4 * i + 1] = b4.y; t[4 * i + 2] = b4.z; t[4 * i + 3] = b4.w;
      }
      if constexpr (BF) {
        // Two taps at a time on v_dot2_f32_bf16: for a channel c the pair
        // (x_a[c], x_b[c]) is gathered from the two taps' words with one
        // v_perm_b32 and dotted with the packed weights (w[c][a], w[c][b]).
        const unsigned* s_w2 = reinterpret_cast<const unsigned*>(s_dw);
        u4 wp[5][2];
#pragma unroll
        for (int pr = 0; pr < 5; ++pr) {
          wp[pr][0] = *reinterpret_cast<const u4*>(s_w2 + pr * cin_pad + ch0);
          wp[pr][1] = *reinterpret_cast<const u4*>(s_w2 + pr * cin_pad + ch0 + 4);
        }
#pragma unroll
        for (int pr = 0; pr < 5; ++pr) {
          Raw ra_ = raw[2 * pr];
          if (!interior && off[2 * pr] < 0) ra_ = Raw{};
          Raw rb_ = Raw{};
          if (pr < 4) {
            rb_ = raw[2 * pr + 1];
            if (!interior && off[2 * pr + 1] < 0) rb_ = Raw{};
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const unsigned p0 = __builtin_amdgcn_perm(ra_[j], rb_[j], 0x01000504u);
            const unsigned p1 = __builtin_amdgcn_perm(ra_[j], rb_[j], 0x03020706u);
            const unsigned w0 = wp[pr][j >> 1][2 * (j & 1)], w1 = wp[pr][j >> 1][2 * (j & 1) + 1];
            t[2 * j] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, p0),
                                                       __builtin_bit_cast(bf16x2, w0), t[2 * j], false);
            t[2 * j + 1] = __builtin_amdgcn_fdot2_f32_bf16(
                __builtin_bit_cast(bf16x2, p1), __builtin_bit_cast(bf16x2, w1), t[2 * j + 1], false);
          }
        }
      } else {
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
          Raw r = raw[tap];
          if (!interior && off[tap] < 0) r = Raw{};
          float v[CH];
          unpack_raw<BF>(r, v);
#pragma unroll
          for (int i = 0; i < CH / 4; ++i) {
            const f4 w4 = s_dw[(tap * cin_pad + ch0) / 4 + i];
            t[4 * i] += w4.x * v[4 * i];
            t[4 * i + 1] += w4.y * v[4 * i + 1];
            t[4 * i + 2] += w4.z * v[4 * i + 2];
            t[4 * i + 3] += w4.w * v[4 * i + 3];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) t[i] = t[i] >= 0.f ? t[i] : a.slope * t[i];
      Frag fa;
      if constexpr (BF)
        fa = u4{pack2(t[0], t[1]), pack2(t[2], t[3]), pack2(t[4], t[5]), pack2(t[6], t[7])};
      else
        fa = f4{t[0], t[1], t[2], t[3]};
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const Frag fb = s_pw[(c * NB + nb) * 64 + lane];
        if constexpr (BF) {
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf8, fa), __builtin_bit_cast(bf8, fb), acc[nb], 0, 0, 0);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[j], fb[j], acc[nb], 0, 0, 0);
        }
      }
    };

    // two tap buffers: chunk c + 1 loads while chunk c computes
    // The fetches are unconditional (past the end they reload the last
    // chunk) so that no branch sits between a load and its use: the wait
    // before each compute then covers only the older buffer.  The
    // scheduling barriers keep the compiler from sinking loads to their use.
    Raw ra[9], rb[9];
    fetch(ra, 0);
    for (int c = 0; c < nchunks; c += 2) {
      fetch(rb, min(c + 1, nchunks - 1));
      __builtin_amdgcn_sched_barrier(0);
      compute(ra, c);
      __builtin_amdgcn_sched_barrier(0);
      fetch(ra, min(c + 2, nchunks - 1));
      __builtin_amdgcn_sched_barrier(0);
      if (c + 1 < nchunks) compute(rb, c + 1);
      __builtin_amdgcn_sched_barrier(0);
    }

    // epilogue: lane holds pixels p0 + 4 lg + v, output channel 16 nb + lm
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int o = nb * 16 + lm;
      if (o >= L.cout) continue;
      const float bo = L.b[o];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = p0 + 4 * lg + v;
        if (p >= hw) continue;
        float r = acc[nb][v] + bo;
        if (a.lrelu) r = r >= 0.f ? r : a.slope * r;
        if (a.add) {
          const size_t q = ((size_t)img * plane + p) * 2 + o;
          reinterpret_cast<float*>(a.out)[q] = a.add[q] + r;
        } else {
          store1(reinterpret_cast<T*>(a.out) +
                     (((size_t)img * a.out_cbt + (o >> 3)) * plane + p) * 8 + (o & 7),
                 r);
        }
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
  if (L.cin_pad * L.np * (L.bf16 ? 2 : 4) > kSepPwFloats * 4) return hipErrorInvalidValue;
  if (a.nblk < 1 || 8 * a.nblk > L.cin_pad || a.nblk > a.in_cbt) return hipErrorInvalidValue;
  if (L.np % 16 || L.np < L.cout || (a.add && L.cout != 2)) return hipErrorInvalidValue;
  const long hw = (long)a.h * a.w;
  if (a.n <= 0 || hw <= 0) return hipSuccess;
  if ((long)a.n * hw > (1L << 30)) return hipErrorInvalidValue;
  // wave tiles of 16 pixels; two resident workgroups per CU
  const long tiles = (long)a.n * ((hw + 15) / 16);
  long groups = (tiles + 3) / 4;
  if (groups > 512) groups = 512;
  return L.bf16 ? dispatch_sep<true>(L, a, dim3((unsigned)groups), s)
                : dispatch_sep<false>(L, a, dim3((unsigned)groups), s);
}

}  // namespace tc
