// 3x3 convolution with FP8 E4M3 operands on gfx950's
// v_mfma_f32_16x16x128_f8f6f4 (K = 128 per instruction, FP32 accumulation).
//
// GEMM view as in the BF16 kernel: M = output pixels, N = output channels,
// K = (tap, 8-channel block) pairs x 8 channels.  One MFMA step consumes 16
// pairs: lane l supplies A[m = l % 16][k = 32 (l / 16) .. + 31], i.e. the 8
// channels of each of the pairs 4 (l / 16) .. 4 (l / 16) + 3 of the step for
// output pixel m, and B the same K range for output channel l % 16.  The
// pairs run tap-major (k = tap * nblk + block) and the last step is padded
// with zero weights, so at most 15 pairs of a layer are wasted.
//
// Workgroup: 4 waves, a (4 MR) x 16 output pixel tile and every output
// channel, as the BF16 kernel.  The input halo of the tile is staged in LDS
// once, with all its channel blocks, converted to FP8 with the image's scale
// max|x| / 448 (inputs stored as bfloat16 or float16); the K loop then only
// streams the weights: one step's 16 pairs x 8 channels x N bytes per stage,
// double-buffered in LDS and fetched four steps ahead into registers, so the
// L2 latency of the weights overlaps several steps of MFMAs (one barrier per
// step).  A per-pair table in
// LDS gives each lane the halo offset of its four pairs (one 16-byte read per
// step).  The epilogue scales the sums back (input scale x per-output-channel
// weight scale), adds the bias, applies LeakyReLU and stores bfloat16 or
// float16 blocks through LDS as whole 16-byte words, and folds the outputs'
// absolute maximum into the image's amax slot when asked.
#include "act.h"
#include "tc_internal.h"

namespace tc {
namespace {

typedef int i8v __attribute__((ext_vector_type(8)));  // 32 bytes: one K = 128 FP8 operand

constexpr int Q8_TW = 16;
constexpr int kF8MaxLds = 64 * 1024;

__host__ __device__ constexpr int al16(int x) { return (x + 15) / 16 * 16; }

template <int S, int MR>
struct F8Geom {
  static constexpr int TH = 4 * MR;
  static constexpr int IH = (TH - 1) * S + 3, IW = (Q8_TW - 1) * S + 3;
  static constexpr int NPOS = IH * IW;
};

__host__ __device__ inline int f8_lds_bytes(int npos, int nblk, int nsteps, int np) {
  return al16(nblk * npos * 8) + al16(nsteps * 16 * 4) + 2 * 4 * np * 32;
}

__device__ inline float f8_amax_of(const AmaxIn& m, int img) {
  const unsigned* p = img < m.nsplit ? m.a : m.b;
  if (!p) return 0.f;
  return read_amax(p + (size_t)(img < m.nsplit ? img : img - m.nsplit) * kAmaxWords);
}

template <typename T>
__device__ inline const T* f8_view_base(const View& v, int img, size_t img_elems) {
  if (v.tab) return reinterpret_cast<const T*>(v.tab[img]);
  return img < v.nsplit ? reinterpret_cast<const T*>(v.a) + (size_t)img * img_elems
                        : reinterpret_cast<const T*>(v.b) + (size_t)(img - v.nsplit) * img_elems;
}

template <int S, int NB, int MR>
__global__ __launch_bounds__(256, 2) void conv3x3_f8k128(ConvArgs a, const unsigned char* __restrict__ w8,
                                                         int nsteps) {
  using G = F8Geom<S, MR>;
  constexpr int TH = G::TH, IW = G::IW, NPOS = G::NPOS;
  constexpr int NP = NB * 16;
  constexpr int WSTEP = 4 * NP * 32;        // bytes of one step's weights
  constexpr int RB = (WSTEP / 16 + 255) / 256;
  constexpr int PD = 4;                     // weight prefetch distance (steps)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int nblk = a.nblk, npairs = 9 * nblk;
  unsigned char* sA = smem;
  int* stab = reinterpret_cast<int*>(smem + al16(nblk * NPOS * 8));
  unsigned char* sB = reinterpret_cast<unsigned char*>(stab) + al16(nsteps * 16 * 4);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  const uint3 tile = xcd_tile();
  const int img = tile.z;
  const int tx0 = tile.x * Q8_TW, ty0 = tile.y * TH;
  const int iy0 = ty0 * S - 1, ix0 = tx0 * S - 1;
  const size_t in_plane = (size_t)a.in_h * a.in_w * 8;

  // Input scale: the stored inputs are the producers' values rounded to
  // bfloat16 or float16, at most 2^-8 above the recorded maximum m in
  // magnitude; the scale is the power of two at or above m (1 + 2^-7) / 448,
  // so every x / sa stays within 448 (the largest lands in (224, 448]) and
  // the scaled conversion applies it exactly.
  float sa = 1.f;
  {
    const float m = fmaxf(f8_amax_of(a.ain[0], img), fmaxf(f8_amax_of(a.ain[1], img), f8_amax_of(a.ain[2], img)));
    if (m > 1.0e-30f && m < 3.0e38f) sa = pow2_ceil(m * (1.f + 0.0078125f) / kFp8Max);
  }

  // The weights of a step are fetched PD steps ahead into a ring of register
  // buffers (slot s % PD) and stored into LDS stage buffer s % 2 one step
  // ahead of use, so their L2 latency overlaps PD - 1 steps of MFMAs.
  u4 rb[PD][RB];
  auto fetch_b = [&](int s, u4 (&r)[RB]) {
    if (s >= nsteps) return;
    const u4* src = reinterpret_cast<const u4*>(w8 + (size_t)s * WSTEP);
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int i = tid + j * 256;
      r[j] = i < WSTEP / 16 ? ldg(src + i) : u4{0u, 0u, 0u, 0u};
    }
  };
  auto stash_b = [&](int b, const u4 (&r)[RB]) {
    u4* dst = reinterpret_cast<u4*>(sB + b * WSTEP);
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int i = tid + j * 256;
      if (i < WSTEP / 16) dst[i] = r[j];
    }
  };
#pragma unroll
  for (int d = 0; d < PD; ++d) fetch_b(d, rb[d]);

  // pair table: halo offset (8-byte words) of pair k = tap * nblk + block;
  // padding pairs point at block 0, tap 0 (their weights are zero)
  for (int k = tid; k < nsteps * 16; k += 256) {
    int off = 0;
    if (k < npairs) {
      const int tap = k / nblk, blk = k - tap * nblk;
      off = blk * NPOS + (tap / 3) * IW + (tap % 3);
    }
    stab[k] = off;
  }

  // the whole input halo, every channel block, as FP8 (zero outside the
  // image): each thread takes halo positions tid, tid + 256, ... and loads
  // every channel block of them (the address math once per position)
  {
    const bf16* base0 = f8_view_base<bf16>(a.in0, img, in_plane * a.in0.cbt);
    const bf16* base1 = f8_view_base<bf16>(a.in1, img, in_plane * a.in1.cbt);
    constexpr int PP = (NPOS + 255) / 256;  // positions per thread
    constexpr int U = 8;                    // blocks loaded together
#pragma unroll
    for (int pp = 0; pp < PP; ++pp) {
      const int pos = tid + pp * 256;
      if (pos >= NPOS) break;
      const int py = pos / IW, px = pos - (pos / IW) * IW;
      const int gy = iy0 + py, gx = ix0 + px;
      const bool in = gy >= 0 && gy < a.in_h && gx >= 0 && gx < a.in_w;
      const size_t off = in ? ((size_t)gy * a.in_w + gx) * 8 : 0;
      for (int b0 = 0; b0 < nblk; b0 += U) {
        u4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int blk = b0 + u;
          v[u] = u4{0u, 0u, 0u, 0u};
          if (in && blk < nblk) {
            const bf16* src = blk < a.nb0 ? base0 + (size_t)(blk + a.in0.cb0) * in_plane
                                          : base1 + (size_t)(blk - a.nb0 + a.in1.cb0) * in_plane;
            v[u] = ldg(reinterpret_cast<const u4*>(src + off));
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int blk = b0 + u;
          if (blk < nblk)
            reinterpret_cast<u2v*>(sA)[blk * NPOS + pos] =
                word_to_fp8_pow2(v[u], (a.in_f16 >> (blk < a.nb0 ? 0 : 1)) & 1, sa);
        }
      }
    }
  }
  stash_b(0, rb[0]);
  fetch_b(PD, rb[0]);
  __syncthreads();

  f4 acc[MR][NB];
#pragma unroll
  for (int i = 0; i < MR; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const u2v* sA8 = reinterpret_cast<const u2v*>(sA);
  auto step = [&](int s, u4 (&rnext)[RB]) {
    const int4 t4 = reinterpret_cast<const int4*>(stab)[s * 4 + lk];
    const int toff[4] = {t4.x, t4.y, t4.z, t4.w};
    const unsigned char* stage = sB + (s & 1) * WSTEP;
    i8v fb[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const u4* q = reinterpret_cast<const u4*>(stage + ((lk * NP + nb * 16 + lm) * 32));
      const u4 lo = q[0], hi = q[1];
      const unsigned w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      fb[nb] = i8v{(int)w[0], (int)w[1], (int)w[2], (int)w[3], (int)w[4], (int)w[5], (int)w[6], (int)w[7]};
    }
#pragma unroll
    for (int mb = 0; mb < MR; ++mb) {
      const int r = wave * MR + mb;
      const int po = r * S * IW + lm * S;
      unsigned w[8];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const u2v x = sA8[toff[j] + po];
        w[2 * j] = x.x;
        w[2 * j + 1] = x.y;
      }
      const i8v fa = i8v{(int)w[0], (int)w[1], (int)w[2], (int)w[3], (int)w[4], (int)w[5], (int)w[6], (int)w[7]};
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fa, fb[nb], acc[mb][nb], 0, 0, 0, 0,
                                                                       0, 0);
    }
    // step s + 1's weights (in slot (s + 1) % PD) into the other stage buffer,
    // then that slot fetches step s + 1 + PD
    if (s + 1 < nsteps) {
      stash_b((s + 1) & 1, rnext);
      fetch_b(s + 1 + PD, rnext);
    }
    __syncthreads();
  };
  for (int s0 = 0; s0 < nsteps; s0 += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d)
      if (s0 + d < nsteps) step(s0 + d, rb[(d + 1) % PD]);
  }

  // epilogue: per output row, each wave writes its 16 x NP results to LDS
  // ([pixel][channel], 16-bit) and stores them back as 16-byte words
  float mx = 0.f;
  bf16* so = reinterpret_cast<bf16*>(smem) + (size_t)wave * (Q8_TW * NP);
  const size_t plane = (size_t)a.out_h * a.out_w;
  // LeakyReLU as max(v, slope v) (0 <= slope <= 1); slope 1 = no activation
  const float slope = a.lrelu ? a.slope : 1.f;
  const bool track = a.aout != nullptr;
  const bool tile_full = tx0 + Q8_TW <= a.out_w && a.cout == NP;  // all columns and channels real
  float osc[NB], bn[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int n = nb * 16 + lm;
    osc[nb] = sa * a.wscale[n];
    bn[nb] = n < a.cout ? a.b[n] : 0.f;
  }
#pragma unroll
  for (int mb = 0; mb < MR; ++mb) {
    const int oy = ty0 + wave * MR + mb;
    wave_lds_sync();  // the wave's own staging region
    float y[NB][4];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const float v = fmaf(acc[mb][nb][vv], osc[nb], bn[nb]);
        y[nb][vv] = fmaxf(v, slope * v);
      }
    if (track && oy < a.out_h) {  // amax of the stored outputs (real channels, in the image)
      if (tile_full) {  // every value of the row is a real output
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int vv = 0; vv < 4; ++vv) mx = fmaxf(mx, fabsf(y[nb][vv]));
      } else {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int vv = 0; vv < 4; ++vv)
            if (nb * 16 + lm < a.cout && tx0 + 4 * lk + vv < a.out_w) mx = fmaxf(mx, fabsf(y[nb][vv]));
      }
    }
    if (a.out_f16) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv)
          so[(4 * lk + vv) * NP + nb * 16 + lm] = __builtin_bit_cast(bf16, (f16)y[nb][vv]);
    } else {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) so[(4 * lk + vv) * NP + nb * 16 + lm] = f2bf(y[nb][vv]);
    }
    wave_lds_sync();  // the wave's own staging region
    if (oy < a.out_h) {
      for (int e = lane; e < Q8_TW * (NP / 8); e += 64) {
        const int px = e / (NP / 8), blk = e - (e / (NP / 8)) * (NP / 8);
        const int ox = tx0 + px;
        if (ox < a.out_w && blk * 8 < a.cout)
          *reinterpret_cast<u4*>(reinterpret_cast<bf16*>(a.out) +
                                 (((size_t)img * a.out_cbt + a.out_cb0 + blk) * plane +
                                  (size_t)oy * a.out_w + ox) * 8) =
              *reinterpret_cast<const u4*>(so + px * NP + blk * 8);
      }
    }
  }
  // every lane of the workgroup reaches this (it reduces across the workgroup)
  if (a.aout) record_amax(a.aout + (size_t)img * kAmaxWords, mx);
}

template <int S, int MR>
hipError_t f8_dispatch(const ConvArgs& a, const unsigned char* w8, int nsteps, hipStream_t s) {
  using G = F8Geom<S, MR>;
  const int lds = f8_lds_bytes(G::NPOS, a.nblk, nsteps, a.np);
  // the epilogue's staging (4 waves x 16 pixels x NP x 2 bytes) fits in the stages
  if (lds > kF8MaxLds || 4 * Q8_TW * a.np * 2 > lds) return hipErrorInvalidValue;
  dim3 grid(cdiv(a.out_w, Q8_TW), cdiv(a.out_h, G::TH), a.n);
  switch (a.np / 16) {
    case 1: conv3x3_f8k128<S, 1, MR><<<grid, 256, lds, s>>>(a, w8, nsteps); break;
    case 2: conv3x3_f8k128<S, 2, MR><<<grid, 256, lds, s>>>(a, w8, nsteps); break;
    case 3: conv3x3_f8k128<S, 3, MR><<<grid, 256, lds, s>>>(a, w8, nsteps); break;
    case 4: conv3x3_f8k128<S, 4, MR><<<grid, 256, lds, s>>>(a, w8, nsteps); break;
    case 5: conv3x3_f8k128<S, 5, MR><<<grid, 256, lds, s>>>(a, w8, nsteps); break;
    case 6: conv3x3_f8k128<S, 6, MR><<<grid, 256, lds, s>>>(a, w8, nsteps); break;
    case 7: conv3x3_f8k128<S, 7, MR><<<grid, 256, lds, s>>>(a, w8, nsteps); break;
    case 8: conv3x3_f8k128<S, 8, MR><<<grid, 256, lds, s>>>(a, w8, nsteps); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int f8k128_steps(int cin_pad) { return cdiv(9 * (cin_pad / 8), 16); }

bool f8k128_ok(const ConvArgs& a, int stride, int mr, int nsteps) {
  if (stride != 1 || a.splits != 1 || a.compact || a.add || !a.fp8 || (mr != 2 && mr != 4))
    return false;
  const int npos = mr == 4 ? F8Geom<1, 4>::NPOS : F8Geom<1, 2>::NPOS;
  return f8_lds_bytes(npos, a.nblk, nsteps, a.np) <= kF8MaxLds && a.np % 16 == 0 && a.np <= 128;
}

hipError_t launch_conv3x3_f8k128(const ConvArgs& a, const void* w8, int nsteps, int mr,
                                 hipStream_t s) {
  if (a.n <= 0 || a.out_h <= 0 || a.out_w <= 0) return hipSuccess;
  if (!w8 || !f8k128_ok(a, 1, mr, nsteps)) return hipErrorInvalidValue;
  const unsigned char* w = static_cast<const unsigned char*>(w8);
  return mr == 4 ? f8_dispatch<1, 4>(a, w, nsteps, s) : f8_dispatch<1, 2>(a, w, nsteps, s);
}

}  // namespace tc
