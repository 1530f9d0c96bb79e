// 3x3 convolution, stride 1, zero padding 1, FP32, by Winograd's minimal
// filtering F(2x2, 3x3) with the element-wise products done as GEMMs on the
// FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Per 2x2 output tile and output channel o:
//   V_c = B^T d_c B          (d_c: the 4x4 input patch of channel c)
//   U_oc = G g_oc G^T        (g_oc: the 3x3 kernel, transformed on the host)
//   M_o = sum_c U_oc (.) V_c (16 independent GEMMs over the input channels)
//   Y_o = A^T M_o A          (the 2x2 outputs)
// with B^T = [1 0 -1 0; 0 1 1 0; 0 -1 1 0; 0 1 0 -1], G = [1 0 0; 1/2 1/2 1/2;
// 1/2 -1/2 1/2; 0 0 1], A^T = [1 1 1 0; 0 1 -1 -1].  The matrix cores then do
// 16 multiplications per tile and channel pair instead of 36 (2.25x fewer);
// every transform is additions and exact halvings, and the sums over input
// channels accumulate in FP32 as in the direct kernel.
//
// Workgroup: 4 waves, a 16 x 16 output pixel tile (8 x 8 Winograd tiles) and
// 32 output channels (two 16-channel N blocks).  Wave w owns the 16 Winograd
// tiles of output rows 4w .. 4w+3.  K runs over chunks of 8 input channels:
// the 18 x 18 input halo of the chunk is staged in LDS (the next chunk is
// prefetched into registers meanwhile, then stored into the second of two
// LDS stage buffers) with the chunk's transformed weights.
// Lane l = 16 g + m transforms the patch of its tile m for channels g and
// g + 4 of the chunk; the 16 values of V are exactly its A operands
// (A[m][k = g]) for the 16 GEMMs, so V never touches LDS.  The accumulators
// of a lane hold all 16 positions of its 4 tiles x 2 channels, so the output
// transform runs in registers; results go through LDS to whole 32-byte
// channel-block stores.
//
// Work mapping: one workgroup per (image, tile row, tile column, channel
// slice), slice fastest, and consecutive work items on the same XCD, so the
// slices that share an input halo run together under one L2.
#include "act.h"
#include "tc_internal.h"

namespace tc {
namespace {

constexpr int WT = 16;             // output tile edge
constexpr int WI = WT + 2;         // input halo edge
constexpr int WNPOS = WI * WI;     // 324 halo pixels
// LDS layout of a staged channel plane: halo rows padded to WRP = 24 floats,
// so the two tile rows a group of 16 lanes reads (2 halo rows apart, 48 =
// 16 mod 32) fall on disjoint banks; planes WAP = 436 floats apart (4 planes
// = 16 mod 32), so the lanes that store channels c and c + 4 of one pixel do
// not collide.
constexpr int WRP = 24;
constexpr int WAP = 436;
constexpr int WNA = WNPOS * 2;     // float4 of input per chunk (8 channels)
constexpr int WRA = (WNA + 255) / 256;
constexpr int WUF = 16 * 2 * 64 * 2;  // transformed weights per chunk and slice
constexpr int WRB = WUF / 4 / 256;
constexpr int WOP = 20;            // epilogue LDS pitch per pixel (16 channels + 4)

__device__ inline const float* wview_base(const View& v, int img, size_t img_floats) {
  if (v.tab) return reinterpret_cast<const float*>(v.tab[img]);
  return img < v.nsplit ? v.a + (size_t)img * img_floats
                        : v.b + (size_t)(img - v.nsplit) * img_floats;
}

__global__ __launch_bounds__(256, 2) void conv3x3_f32_wino(ConvArgs a, const float* __restrict__ wu,
                                                           int nsl, int gx, int gy, int total) {
  // two stage buffers (input halo + transformed weights of one chunk each):
  // chunk c + 1 is stored into one while the matrix cores consume the other
  constexpr int STAGE = 8 * WAP + WUF;
  __shared__ __attribute__((aligned(16))) float smem[2 * STAGE];

  // XCD-aware work id: block b runs on XCD b % 8; give each XCD a contiguous
  // range of work ids (a bijection of [0, total)).
  const int bid = blockIdx.x;
  const int q = total / 8, r = total % 8, x = bid % 8;
  const int wid = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + bid / 8;
  const int sl = wid % nsl;
  int t = wid / nsl;
  const int tcx = t % gx;
  t /= gx;
  const int tcy = t % gy;
  const int img = t / gy;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  const int tx0 = tcx * WT, ty0 = tcy * WT;
  const int iy0 = ty0 - 1, ix0 = tx0 - 1;
  const size_t in_plane = (size_t)a.in_h * a.in_w * 8;
  const float* wslice = wu + (size_t)sl * a.nchunks * WUF;

  f4 acc[16][2];
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    acc[p][0] = f4{0.f, 0.f, 0.f, 0.f};
    acc[p][1] = f4{0.f, 0.f, 0.f, 0.f};
  }

  // Prefetch of a chunk: every load is unconditional (addresses clamped into
  // the image, the same for every chunk, so computed once) and no branch
  // join makes the compiler wait for them; the zero padding is applied when
  // the values are stored into LDS.
  f4 ra[WRA], rb[WRB];
  int off[WRA];      // float offset of ra[j] within a channel block
  unsigned inb = 0;  // bit j: ra[j] is inside the image
#pragma unroll
  for (int j = 0; j < WRA; ++j) {
    const int i = tid + j * 256;
    const int ic = i < WNA ? i : WNA - 1;
    const int pos = ic >> 1, c4 = ic & 1;
    const int py = pos / WI, px = pos - py * WI;
    const int gy_ = iy0 + py, gx_ = ix0 + px;
    const bool ok = i < WNA && gy_ >= 0 && gy_ < a.in_h && gx_ >= 0 && gx_ < a.in_w;
    const int cy = min(max(gy_, 0), a.in_h - 1), cx = min(max(gx_, 0), a.in_w - 1);
    off[j] = (cy * a.in_w + cx) * 8 + c4 * 4;
    inb |= (ok ? 1u : 0u) << j;
  }
  auto fetch = [&](int ch) {
    const View& v = ch < a.nb0 ? a.in0 : a.in1;
    const int cb = (ch < a.nb0 ? ch : ch - a.nb0) + v.cb0;
    const float* src = wview_base(v, img, in_plane * v.cbt) + (size_t)cb * in_plane;
#pragma unroll
    for (int j = 0; j < WRA; ++j) ra[j] = ldg(reinterpret_cast<const f4*>(src + off[j]));
    const f4* ws = reinterpret_cast<const f4*>(wslice + (size_t)ch * WUF);
#pragma unroll
    for (int j = 0; j < WRB; ++j) rb[j] = ldg(ws + tid + j * 256);
  };
  auto stash = [&](float* st) {
#pragma unroll
    for (int j = 0; j < WRA; ++j) {
      const int i = tid + j * 256;
      if (i < WNA) {
        const int pos = i >> 1, c4 = i & 1;
        const f4 val = ((inb >> j) & 1u) ? ra[j] : f4{0.f, 0.f, 0.f, 0.f};
        const int py = pos / WI, lp = py * WRP + (pos - py * WI);
        st[(c4 * 4 + 0) * WAP + lp] = val.x;
        st[(c4 * 4 + 1) * WAP + lp] = val.y;
        st[(c4 * 4 + 2) * WAP + lp] = val.z;
        st[(c4 * 4 + 3) * WAP + lp] = val.w;
      }
    }
#pragma unroll
    for (int j = 0; j < WRB; ++j) reinterpret_cast<f4*>(st + 8 * WAP)[tid + j * 256] = rb[j];
  };

  // this lane's Winograd tile (A row m = lm): tile row 2 * wave + lm / 8, column lm % 8
  const int aoff = 2 * (2 * wave + (lm >> 3)) * WRP + 2 * (lm & 7);

  // the 4x4 patch of channel c of the lane's tile, and its transform B^T d B
  auto read_patch = [&](const float* st, int c, float (&d)[16]) {
    const float* s = st + c * WAP + aoff;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float2 lo = *reinterpret_cast<const float2*>(s + i * WRP);
      const float2 hi = *reinterpret_cast<const float2*>(s + i * WRP + 2);
      d[4 * i + 0] = lo.x;
      d[4 * i + 1] = lo.y;
      d[4 * i + 2] = hi.x;
      d[4 * i + 3] = hi.y;
    }
  };
  auto transform = [&](const float (&d)[16], float (&v)[16]) {
    float rr[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      rr[0][j] = d[j] - d[8 + j];
      rr[1][j] = d[4 + j] + d[8 + j];
      rr[2][j] = d[8 + j] - d[4 + j];
      rr[3][j] = d[4 + j] - d[12 + j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[4 * i + 0] = rr[i][0] - rr[i][2];
      v[4 * i + 1] = rr[i][1] + rr[i][2];
      v[4 * i + 2] = rr[i][2] - rr[i][1];
      v[4 * i + 3] = rr[i][1] - rr[i][3];
    }
  };

  const int c_end = a.nchunks;
  fetch(0);
  stash(smem);
  __syncthreads();
  for (int ch = 0; ch < c_end; ++ch) {
    const float* st = smem + (ch & 1) * STAGE;
    if (ch + 1 < c_end) fetch(ch + 1);
    const float* sUl = st + 8 * WAP + lane * 2;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      // all LDS reads of the step first (the patch and the 16 B fragments),
      // then the transform, then the 32 MFMAs back to back
      float d[16], v[16];
      float2 u[16];
      read_patch(st, 4 * ks + lk, d);
#pragma unroll
      for (int p = 0; p < 16; ++p) u[p] = *reinterpret_cast<const float2*>(sUl + (ks * 16 + p) * 128);
      transform(d, v);
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        acc[p][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[p], u[p].x, acc[p][0], 0, 0, 0);
        acc[p][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[p], u[p].y, acc[p][1], 0, 0, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x100, 24, 0);  // 8 patch + 16 fragment reads
      __builtin_amdgcn_sched_group_barrier(0x002, 32, 0);  // the transform
      __builtin_amdgcn_sched_group_barrier(0x008, 32, 0);  // the MFMAs
    }
    if (ch + 1 < c_end) stash(smem + ((ch + 1) & 1) * STAGE);
    __syncthreads();
  }

  // ---- output transform, bias, LeakyReLU; through LDS to 32-byte block stores
  float* so = smem + wave * (64 * WOP);
  const size_t plane = (size_t)a.out_h * a.out_w;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int n = sl * 32 + nb * 16 + lm;  // output channel of this lane
    const float bn = n < a.cout ? a.b[n] : 0.f;
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int m = 4 * lk + vv;  // tile within the wave
      float M[4][4];
#pragma unroll
      for (int p = 0; p < 16; ++p) M[p >> 2][p & 3] = acc[p][nb][vv];
      float tt[2][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        tt[0][j] = M[0][j] + M[1][j] + M[2][j];
        tt[1][j] = M[1][j] - M[2][j] - M[3][j];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        float y0 = tt[i][0] + tt[i][1] + tt[i][2] + bn;
        float y1 = tt[i][1] - tt[i][2] - tt[i][3] + bn;
        if (a.lrelu) {
          y0 = y0 >= 0.f ? y0 : a.slope * y0;
          y1 = y1 >= 0.f ? y1 : a.slope * y1;
        }
        const int lr = 2 * (m >> 3) + i;  // row within the wave's 4 output rows
        const int lc = 2 * (m & 7);
        so[(lr * WT + lc) * WOP + lm] = y0;
        so[(lr * WT + lc + 1) * WOP + lm] = y1;
      }
    }
    wave_lds_sync();  // the wave's own staging region
    // 64 pixels x 2 blocks of 8 channels per wave
#pragma unroll
    for (int e = lane; e < 128; e += 64) {
      const int px = e >> 1, blk = e & 1;
      const int oy = ty0 + 4 * wave + (px >> 4), ox = tx0 + (px & 15);
      const int cblk = (sl * 32 + nb * 16) / 8 + blk;
      if (oy < a.out_h && ox < a.out_w && cblk * 8 < a.cout) {
        const f4* src = reinterpret_cast<const f4*>(so + px * WOP + blk * 8);
        f4* dst = reinterpret_cast<f4*>(
            a.out + (((size_t)img * a.out_cbt + a.out_cb0 + cblk) * plane + (size_t)oy * a.out_w + ox) * 8);
        dst[0] = src[0];
        dst[1] = src[1];
      }
    }
    wave_lds_sync();  // the wave's own staging region
  }
}

}  // namespace

bool wino_ok(const ConvArgs& a, int stride, int kc) {
  return stride == 1 && kc == 8 && !a.bf16act && !a.fp8 && !a.compact && !a.add &&
         a.np % 32 == 0 && a.cout % 8 == 0 && a.in_h == a.out_h && a.in_w == a.out_w;
}

hipError_t launch_conv3x3_wino(const ConvArgs& a, const float* wu, hipStream_t s) {
  if (a.n <= 0 || a.out_h <= 0 || a.out_w <= 0) return hipSuccess;
  if (!wu || !wino_ok(a, 1, 8)) return hipErrorInvalidValue;
  const int nsl = a.np / 32;
  const int gx = cdiv(a.out_w, WT), gy = cdiv(a.out_h, WT);
  const long total = (long)nsl * gx * gy * a.n;
  if (total > 0x7fffffffL) return hipErrorInvalidValue;
  conv3x3_f32_wino<<<(unsigned)total, 256, 0, s>>>(a, wu, nsl, gx, gy, (int)total);
  return hipGetLastError();
}

// U = G g G^T per (output, input) channel pair, in double, rounded once to
// float; packed per 32-channel output slice and chunk of 8 input channels as
// [slice][chunk][ks (2)][position (16)][lane (64)][N block (2)], the value of
// lane 16 g + m being U[position][input 8 chunk + 4 ks + g][output 32 slice +
// 16 block + m].  cmap maps packed input channels to source channels (-1 =
// zero).
void pack_conv_wino(const float* W, int cout, int cin, int cin_pad, const std::vector<int>& cmap,
                    std::vector<float>& out) {
  const int np = cdiv(cout, 32) * 32, nsl = np / 32, nch = cin_pad / 8;
  out.assign((size_t)nsl * nch * WUF, 0.f);
  for (int o = 0; o < cout; ++o) {
    const int sl = o / 32, nb = (o % 32) / 16, m = o % 16;
    for (int gch = 0; gch < cin_pad; ++gch) {
      const int c = cmap[gch];
      if (c < 0) continue;
      const float* g = W + ((size_t)o * cin + c) * 9;
      double Gg[4][3], U[4][4];
      for (int j = 0; j < 3; ++j) {
        const double g0 = g[j], g1 = g[3 + j], g2 = g[6 + j];
        Gg[0][j] = g0;
        Gg[1][j] = 0.5 * (g0 + g1 + g2);
        Gg[2][j] = 0.5 * (g0 - g1 + g2);
        Gg[3][j] = g2;
      }
      for (int i = 0; i < 4; ++i) {
        U[i][0] = Gg[i][0];
        U[i][1] = 0.5 * (Gg[i][0] + Gg[i][1] + Gg[i][2]);
        U[i][2] = 0.5 * (Gg[i][0] - Gg[i][1] + Gg[i][2]);
        U[i][3] = Gg[i][2];
      }
      const int chunk = gch / 8, kk = gch % 8, ks = kk / 4, gg = kk % 4;
      const int lane = 16 * gg + m;
      for (int p = 0; p < 16; ++p)
        out[(((((size_t)sl * nch + chunk) * 2 + ks) * 16 + p) * 64 + lane) * 2 + nb] =
            (float)U[p >> 2][p & 3];
    }
  }
}

}  // namespace tc
