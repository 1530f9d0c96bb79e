// 3x3 convolution, stride 1, zero padding 1, FP32, by Winograd's minimal
// filtering F(4x4, 3x3) with the element-wise products done as GEMMs on the
// FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// Per 4x4 output tile and output channel o (Lavin and Gray's construction):
//   V_c = B^T d_c B          (d_c: the 6x6 input patch of channel c)
//   U_oc = G g_oc G^T        (g_oc: the 3x3 kernel, transformed on the host)
//   M_o = sum_c U_oc (.) V_c (36 independent GEMMs over the input channels)
//   Y_o = A^T M_o A          (the 4x4 outputs)
// with
//   B^T = [4 0 -5 0 1 0; 0 -4 -4 1 1 0; 0 4 -4 -1 1 0; 0 -2 -1 2 1 0;
//          0 2 -1 -2 1 0; 0 4 0 -5 0 1]
//   G   = [1/4 0 0; -1/6 -1/6 -1/6; -1/6 1/6 -1/6; 1/24 1/12 1/6;
//          1/24 -1/12 1/6; 0 0 1]
//   A^T = [1 1 1 1 1 0; 0 1 -1 2 -2 0; 0 1 1 4 4 0; 0 1 -1 8 -8 1].
// The matrix cores do 36 multiplications per tile and channel pair instead of
// direct convolution's 144 (4x fewer; F(2x2, 3x3) does 64 per 4x4 outputs).
// The transforms are FP32 additions and multiplications by small integers;
// G's fractions are applied to the weights in double on the host, rounded
// once.  The larger transform coefficients cost accuracy: a few times FP32
// rounding per term, far inside the flow tolerance.
//
// Workgroup: 4 waves, a 16 x 32 output pixel region (4 x 8 Winograd tiles)
// and 32 output channels.  Wave w owns M block w / 2 (tile rows 2 (w/2) and
// 2 (w/2) + 1: 16 tiles) and N block w % 2 (16 channels).  K runs over
// chunks of 4 input channels (one MFMA K step): the 18 x 34 input halo of the
// chunk is staged in one of two LDS stage buffers while the matrix cores
// consume the other (the next chunk is prefetched into registers meanwhile).
// Lane l = 16 g + m transforms the 6x6 patch of tile m for channel g: its 36
// values are exactly its A operands (A[m][k = g]) for the 36 GEMMs, so V
// never touches LDS.  Its 36 B operands (the transformed weights of input g
// and output m of its N block) are 144 contiguous bytes of the chunk's
// 18 KB of transformed weights, which travel from global memory straight
// into a second pair of LDS buffers (direct global-to-LDS loads, one chunk
// ahead, no registers): the two waves of an N block read one copy.  A chunk
// reads all its LDS operands first and only then issues the next chunk's
// loads, so the matrix instructions never wait on memory.  The accumulators
// of a lane hold all 36 positions of its 4 tiles, so the output transform
// runs in registers; results go through LDS to whole 32-byte channel-block
// stores.
//
// Work mapping: one workgroup per (image, region row, region column, channel
// slice), slice fastest, consecutive work items on the same XCD, so the
// slices that share an input halo run together under one L2.
#include "act.h"
#include "tc_internal.h"

namespace tc {
namespace {

// QM = M blocks (pairs of tile rows, 8 output rows) per workgroup; the
// workgroup has 2 QM waves (one per M block and 16-channel N block).
template <int QM>
struct Q4 {
  static constexpr int THREADS = 128 * QM;
  static constexpr int QY = 8 * QM, QX = 32;           // output rows and columns
  static constexpr int QHY = QY + 2, QHX = QX + 2;     // input halo
  // LDS row pitch of a staged plane (floats): 40, so the tiles of the two
  // tile rows of an M block (4 halo rows apart: 160 floats = 32 mod 64)
  // read disjoint banks
  static constexpr int QRP = 40;
  static constexpr int QAP = QHY * QRP + 8;            // LDS plane pitch (= 16 mod 32)
  static constexpr int QNA = QHY * QHX;                // halo pixels, one float4 (4 channels) each
  static constexpr int QRA = (QNA + THREADS - 1) / THREADS;
  static constexpr int QSTAGE = 4 * QAP;               // floats per stage buffer (halo only)
};
constexpr int QUF = 2 * 64 * 36;  // transformed weights per chunk and 32-channel slice
constexpr int QOP = 20;  // epilogue LDS pitch per pixel (16 channels + 4)

__device__ inline const float* qview_base(const View& v, int img, size_t img_floats) {
  if (v.tab) return reinterpret_cast<const float*>(v.tab[img]);
  return img < v.nsplit ? v.a + (size_t)img * img_floats
                        : v.b + (size_t)(img - v.nsplit) * img_floats;
}

// y = B^T x for one 6-vector
__device__ inline void bt6(const float (&x)[6], float (&y)[6]) {
  const float t0 = fmaf(-4.f, x[2], x[4]);  // x4 - 4 x2
  const float t1 = fmaf(-4.f, x[1], x[3]);  // x3 - 4 x1
  const float t2 = x[4] - x[2];
  const float t3 = 2.f * (x[3] - x[1]);
  y[0] = fmaf(4.f, x[0], fmaf(-5.f, x[2], x[4]));
  y[1] = t0 + t1;
  y[2] = t0 - t1;
  y[3] = t2 + t3;
  y[4] = t2 - t3;
  y[5] = fmaf(4.f, x[1], fmaf(-5.f, x[3], x[5]));
}

// z = A^T x for one 6-vector
__device__ inline void at6(const float (&x)[6], float (&z)[4]) {
  const float s1 = x[1] + x[2], d1 = x[1] - x[2];
  const float s2 = x[3] + x[4], d2 = x[3] - x[4];
  z[0] = x[0] + s1 + s2;
  z[1] = fmaf(2.f, d2, d1);
  z[2] = fmaf(4.f, s2, s1);
  z[3] = fmaf(8.f, d2, d1) + x[5];
}

template <int QM>
__global__ __launch_bounds__(128 * QM, 4 / QM) void conv3x3_f32_wino4(ConvArgs a, const float* __restrict__ wu,
                                                                     int nsl, int gx, int gy, int total) {
  using C = Q4<QM>;
  constexpr int THREADS = C::THREADS, QY = C::QY, QX = C::QX, QHX = C::QHX, QRP = C::QRP,
                QAP = C::QAP, QNA = C::QNA, QRA = C::QRA,
                QSTAGE = C::QSTAGE;
  // Two transformed-weight buffers and two halo stage buffers, as separate
  // arrays: the compiler can then tell the weights' direct LDS loads from
  // the halo reads and does not wait for those loads before every read.
  // After the K loop the weight buffers hold the epilogue's 64 pixels x QOP
  // per wave.
  static_assert(2 * QM * 64 * QOP <= 2 * QUF, "epilogue exceeds the weight buffers");
  __shared__ __attribute__((aligned(16))) float ubuf[2 * QUF];
  __shared__ __attribute__((aligned(16))) float stage[2 * QSTAGE];

  // XCD-aware work id: block b runs on XCD b % 8; give each XCD a contiguous
  // range of work ids (a bijection of [0, total)).
  const int bid = blockIdx.x;
  const int q = total / 8, r = total % 8, xc = bid % 8;
  const int wid = (xc < r ? xc * (q + 1) : r * (q + 1) + (xc - r) * q) + bid / 8;
  const int sl = wid % nsl;
  int t = wid / nsl;
  const int tcx = t % gx;
  t /= gx;
  const int tcy = t % gy;
  const int img = t / gy;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lm = lane & 15, lg = lane >> 4;
  const int mblk = wave >> 1, nb = wave & 1;
  const int tx0 = tcx * QX, ty0 = tcy * QY;
  const int iy0 = ty0 - 1, ix0 = tx0 - 1;
  const size_t in_plane = (size_t)a.in_h * a.in_w * 8;
  const int nch = a.nblk * 2;  // chunks of 4 input channels
  const float* wslice = wu + (size_t)sl * nch * QUF;

  f4 acc[36];
#pragma unroll
  for (int p = 0; p < 36; ++p) acc[p] = f4{0.f, 0.f, 0.f, 0.f};

  // Prefetch of a chunk: unconditional loads (addresses clamped into the
  // image, the same for every chunk, so computed once); the zero padding is
  // applied when the values are stored into LDS.
  f4 ra[QRA];
  int off[QRA];
  unsigned inb = 0;
#pragma unroll
  for (int j = 0; j < QRA; ++j) {
    const int i = tid + j * THREADS;
    const int ic = i < QNA ? i : QNA - 1;
    const int py = ic / QHX, px = ic - py * QHX;
    const int gy_ = iy0 + py, gx_ = ix0 + px;
    const bool ok = i < QNA && gy_ >= 0 && gy_ < a.in_h && gx_ >= 0 && gx_ < a.in_w;
    const int cy = min(max(gy_, 0), a.in_h - 1), cx = min(max(gx_, 0), a.in_w - 1);
    off[j] = (cy * a.in_w + cx) * 8;
    inb |= (ok ? 1u : 0u) << j;
  }
  // the two input views' image bases, read once (a view may hold a table
  // of per-image pointers)
  const float* const base0 = qview_base(a.in0, img, in_plane * a.in0.cbt) + (size_t)a.in0.cb0 * in_plane;
  const float* const base1 =
      a.nblk > a.nb0 ? qview_base(a.in1, img, in_plane * a.in1.cbt) + (size_t)a.in1.cb0 * in_plane : base0;
  auto fetch = [&](int ch) {
    const int b = ch >> 1;
    const float* src = (b < a.nb0 ? base0 + (size_t)b * in_plane : base1 + (size_t)(b - a.nb0) * in_plane) +
                       (ch & 1) * 4;
#pragma unroll
    for (int j = 0; j < QRA; ++j) ra[j] = ldg(reinterpret_cast<const f4*>(src + off[j]));
  };
  auto stash = [&](float* st) {
#pragma unroll
    for (int j = 0; j < QRA; ++j) {
      const int i = tid + j * THREADS;
      if (i < QNA) {
        const int py = i / QHX, px = i - py * QHX;
        const f4 val = ((inb >> j) & 1u) ? ra[j] : f4{0.f, 0.f, 0.f, 0.f};
        const int lp = py * QRP + px;
        st[0 * QAP + lp] = val.x;
        st[1 * QAP + lp] = val.y;
        st[2 * QAP + lp] = val.z;
        st[3 * QAP + lp] = val.w;
      }
    }
  };

  // The chunk's transformed weights (QUF floats = 18 pieces of 1 KB) go
  // straight from global memory into an LDS buffer (global_load_lds: lane l
  // of a wave writes bytes 16 l .. 16 l + 15 of the wave's 1 KB piece), one
  // chunk ahead of their use, without passing through registers.  Wave w
  // loads pieces w, w + 4, ... (THREADS / 64 waves share the 18 pieces).
  constexpr int NWAVE = THREADS / 64, UPIECES = QUF / 256;
  auto fetch_u = [&](int ch, float* dst) {
    const float* src = wslice + (size_t)ch * QUF + lane * 4;
#pragma unroll
    for (int kb = wave; kb < UPIECES; kb += NWAVE)
      __builtin_amdgcn_global_load_lds(
          reinterpret_cast<const void*>(src + kb * 256),
          (__attribute__((address_space(3))) void*)(dst + kb * 256), 16, 0, 0);
  };

  // this lane's tile (A row m = lm): tile row 2 mblk + lm / 8, column lm % 8;
  // its patch in channel plane lg
  const int aoff = lg * QAP + 4 * (2 * mblk + (lm >> 3)) * QRP + 4 * (lm & 7);
  // its 36 transformed weights (B[k = lg][n = lm] of every position)
  const int uoff = (nb * 64 + lane) * 36;

  fetch_u(0, ubuf);
  fetch(0);
  stash(stage);
  __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0) (the weights' LDS loads) and lgkmcnt(0)
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const float* st = stage + (ch & 1) * QSTAGE;
    // All of the chunk's LDS reads come first: the compiler orders LDS reads
    // after a pending direct LDS load behind a wait for it, so the next
    // chunk's loads are issued only once this chunk's operands are read.
    f4 uq[9];
    {
      const f4* up = reinterpret_cast<const f4*>(ubuf + (ch & 1) * QUF + uoff);
#pragma unroll
      for (int k = 0; k < 9; ++k) uq[k] = up[k];
    }
    // the patch, then V = B^T d B (columns first, then rows)
    float d[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const f4 lo = *reinterpret_cast<const f4*>(st + aoff + i * QRP);
      const float2 hi = *reinterpret_cast<const float2*>(st + aoff + i * QRP + 4);
      d[i][0] = lo.x;
      d[i][1] = lo.y;
      d[i][2] = lo.z;
      d[i][3] = lo.w;
      d[i][4] = hi.x;
      d[i][5] = hi.y;
    }
    if (ch + 1 < nch) {
      fetch(ch + 1);
      fetch_u(ch + 1, ubuf + ((ch + 1) & 1) * QUF);
    }
    float tcol[6][6];  // tcol[p][j] = (B^T d)[p][j]
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const float x[6] = {d[0][j], d[1][j], d[2][j], d[3][j], d[4][j], d[5][j]};
      float y[6];
      bt6(x, y);
#pragma unroll
      for (int p = 0; p < 6; ++p) tcol[p][j] = y[p];
    }
    float v[36];
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      float y[6];
      bt6(tcol[p], y);
#pragma unroll
      for (int qq = 0; qq < 6; ++qq) v[6 * p + qq] = y[qq];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const f4 u = uq[k];
      acc[4 * k + 0] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[4 * k + 0], u.x, acc[4 * k + 0], 0, 0, 0);
      acc[4 * k + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[4 * k + 1], u.y, acc[4 * k + 1], 0, 0, 0);
      acc[4 * k + 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[4 * k + 2], u.z, acc[4 * k + 2], 0, 0, 0);
      acc[4 * k + 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[4 * k + 3], u.w, acc[4 * k + 3], 0, 0, 0);
    }
    if (ch + 1 < nch) stash(stage + ((ch + 1) & 1) * QSTAGE);
    __builtin_amdgcn_s_waitcnt(0);  // the next chunk's weights have landed in LDS
    __syncthreads();
  }

  // ---- output transform, bias, LeakyReLU; through LDS to 32-byte block
  // stores.  Lane (lg, lm) holds tiles 4 lg + vv (vv = 0..3) of its M block
  // for output channel sl * 32 + nb * 16 + lm.  Four passes of 4 tiles each
  // (vv = pass); tile k of a pass is 4 k + pass.
  float* so = ubuf + wave * (64 * QOP);
  const size_t plane = (size_t)a.out_h * a.out_w;
  const int n = sl * 32 + nb * 16 + lm;
  const float bn = n < a.cout ? a.b[n] : 0.f;
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    {
      const int vv = pass;
      float tc4[4][6];  // (A^T M)[i][qq]
#pragma unroll
      for (int qq = 0; qq < 6; ++qq) {
        const float x[6] = {acc[qq][vv], acc[6 + qq][vv], acc[12 + qq][vv], acc[18 + qq][vv],
                            acc[24 + qq][vv], acc[30 + qq][vv]};
        float z[4];
        at6(x, z);
#pragma unroll
        for (int i = 0; i < 4; ++i) tc4[i][qq] = z[i];
      }
      const int k = lg;  // tile of the pass
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float z[4];
        at6(tc4[i], z);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          float y = z[jj] + bn;
          if (a.lrelu) y = y >= 0.f ? y : a.slope * y;
          so[(k * 16 + i * 4 + jj) * QOP + lm] = y;
        }
      }
    }
    wave_lds_sync();  // the wave's own staging region
    // 64 pixels x 2 blocks of 8 channels per wave
#pragma unroll
    for (int e = lane; e < 128; e += 64) {
      const int px = e >> 1, blk = e & 1;
      const int k = px >> 4, i = (px >> 2) & 3, jj = px & 3;
      const int tile = 4 * k + pass;
      const int oy = ty0 + 4 * (2 * mblk + (tile >> 3)) + i;
      const int ox = tx0 + 4 * (tile & 7) + jj;
      const int cblk = (sl * 32 + nb * 16) / 8 + blk;
      if (oy < a.out_h && ox < a.out_w && cblk * 8 < a.cout) {
        const f4* src = reinterpret_cast<const f4*>(so + px * QOP + blk * 8);
        f4* dst = reinterpret_cast<f4*>(
            a.out + (((size_t)img * a.out_cbt + a.out_cb0 + cblk) * plane + (size_t)oy * a.out_w + ox) * 8);
        dst[0] = src[0];
        dst[1] = src[1];
      }
    }
    wave_lds_sync();  // the wave's own staging region
  }
}

constexpr int kWino4M = 2;

}  // namespace

hipError_t launch_conv3x3_wino4(const ConvArgs& a, const float* wu4, hipStream_t s) {
  if (a.n <= 0 || a.out_h <= 0 || a.out_w <= 0) return hipSuccess;
  if (!wu4 || !wino_ok(a, 1, 8)) return hipErrorInvalidValue;
  constexpr int QM = kWino4M;
  const int nsl = a.np / 32;
  const int gx = cdiv(a.out_w, Q4<QM>::QX), gy = cdiv(a.out_h, Q4<QM>::QY);
  const long total = (long)nsl * gx * gy * a.n;
  if (total > 0x7fffffffL) return hipErrorInvalidValue;
  conv3x3_f32_wino4<QM><<<(unsigned)total, Q4<QM>::THREADS, 0, s>>>(a, wu4, nsl, gx, gy, (int)total);
  return hipGetLastError();
}

// U = G g G^T per (output, input) channel pair, in double, rounded once to
// float; packed per 32-channel output slice and chunk of 4 input channels as
// [slice][chunk][N block (2)][lane (64)][position (36)], the value of lane
// 16 g + m being U[position][input 4 chunk + g][output 32 slice + 16 block +
// m].  cmap maps packed input channels to source channels (-1 = zero).
void pack_conv_wino4(const float* W, int cout, int cin, int cin_pad, const std::vector<int>& cmap,
                     std::vector<float>& out) {
  static const double G[6][3] = {{1.0 / 4, 0.0, 0.0},
                                 {-1.0 / 6, -1.0 / 6, -1.0 / 6},
                                 {-1.0 / 6, 1.0 / 6, -1.0 / 6},
                                 {1.0 / 24, 1.0 / 12, 1.0 / 6},
                                 {1.0 / 24, -1.0 / 12, 1.0 / 6},
                                 {0.0, 0.0, 1.0}};
  const int np = cdiv(cout, 32) * 32, nsl = np / 32, nch = cin_pad / 4;
  out.assign((size_t)nsl * nch * QUF, 0.f);
  for (int o = 0; o < cout; ++o) {
    const int sl = o / 32, nbk = (o % 32) / 16, m = o % 16;
    for (int gch = 0; gch < cin_pad; ++gch) {
      const int c = cmap[gch];
      if (c < 0) continue;
      const float* g = W + ((size_t)o * cin + c) * 9;
      double Gg[6][3], U[6][6];
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 3; ++j)
          Gg[i][j] = G[i][0] * g[j] + G[i][1] * g[3 + j] + G[i][2] * g[6 + j];
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) U[i][j] = Gg[i][0] * G[j][0] + Gg[i][1] * G[j][1] + Gg[i][2] * G[j][2];
      const int chunk = gch / 4, gg = gch % 4;
      const int lane = 16 * gg + m;
      for (int p = 0; p < 36; ++p)
        out[((((size_t)sl * nch + chunk) * 2 + nbk) * 64 + lane) * 36 + p] = (float)U[p / 6][p % 6];
    }
  }
}

}  // namespace tc
