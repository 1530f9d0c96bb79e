// The paper's full consistency step (Sec. 3.1): local and global consistency
// references and weights (Eq. 2-7), then the screened-Poisson energy (Eq. 1)
// minimised by gradient descent with momentum (Eq. 8).
//
// With R = w_c A - Lap(P) precomputed, the gradient of the discrete energy is
//   grad E(O) = -Lap(O) + w_c O - R
// (5-point Laplacian, Neumann borders), and one iteration is
//   O' = O - eta grad E(O) + kappa (O - O_old).
// The iterations are temporally blocked: a workgroup loads a 64 x 48 region
// (wave w a 64 x 12 strip, one column per lane, its 12 rows in registers),
// takes the horizontal neighbours by DPP wave shifts, the vertical ones from
// its own registers and, at a strip's first and last row, from the
// neighbouring strip through LDS, and runs K iterations (7 per pass); after
// K iterations the region's border of width K holds stale values and only
// the interior (64 - 2K) x (48 - 2K) is written back.  Border pixels of the
// image use only their in-image neighbours.  Regions run in XCD-aware order,
// so the overlapping borders of neighbouring regions are read into one L2.
#include "tc_internal.h"

namespace tc {
namespace {

struct Tap {
  int o00, o01, o10, o11;
  float w00, w01, w10, w11;
};

// Bilinear taps of x + f, indices clamped to the image (border value); the
// integer part comes from the flow alone so the weights are exact.
__device__ inline Tap taps(int x, int y, float fx, float fy, int w, int h) {
  const float bx = floorf(fx), by = floorf(fy);
  const float ax = fx - bx, ay = fy - by;
  const int ix = (int)fminf(fmaxf((float)x + bx, -2.f), (float)w + 1.f);
  const int iy = (int)fminf(fmaxf((float)y + by, -2.f), (float)h + 1.f);
  const int x0 = min(max(ix, 0), w - 1), x1 = min(max(ix + 1, 0), w - 1);
  const int y0 = min(max(iy, 0), h - 1), y1 = min(max(iy + 1, 0), h - 1);
  Tap t;
  t.o00 = y0 * w + x0;
  t.o01 = y0 * w + x1;
  t.o10 = y1 * w + x0;
  t.o11 = y1 * w + x1;
  t.w00 = (1.f - ax) * (1.f - ay);
  t.w01 = ax * (1.f - ay);
  t.w10 = (1.f - ax) * ay;
  t.w11 = ax * ay;
  return t;
}

__device__ inline float sample(const float* p, const Tap& t) {
  return t.w00 * p[t.o00] + t.w01 * p[t.o01] + t.w10 * p[t.o10] + t.w11 * p[t.o11];
}

__global__ __launch_bounds__(256) void paper_reference_kernel(PaperArgs a) {
  const size_t plane = (size_t)a.h * a.w;
  const size_t total = (size_t)a.n * plane;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t img = i / plane, pix = i - img * plane;
    const int y = (int)(pix / a.w), x = (int)(pix - (size_t)y * a.w);
    const size_t o3 = img * 3 * plane, o2 = img * 2 * plane;
    const Tap tp = taps(x, y, a.f_tp[o2 + pix], a.f_tp[o2 + plane + pix], a.w, a.h);
    const Tap tn = taps(x, y, a.f_tn[o2 + pix], a.f_tn[o2 + plane + pix], a.w, a.h);
    float I[3], Ip[3], In[3], P[3], Pp[3], Pn[3], G[3];
    float dp = 0.f, dn = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t oc = o3 + c * plane;
      I[c] = a.I[oc + pix];
      P[c] = a.P[oc + pix];
      Ip[c] = sample(a.I_prev + oc, tp);
      Pp[c] = sample(a.P_prev + oc, tp);
      G[c] = sample(a.O_prev + oc, tp);
      In[c] = sample(a.I_next + oc, tn);
      Pn[c] = sample(a.P_next + oc, tn);
      dp += (I[c] - Ip[c]) * (I[c] - Ip[c]);
      dn += (I[c] - In[c]) * (I[c] - In[c]);
    }
    const float wp = fminf(expf(-a.a_ph * dp), a.k1);
    const float wn = fminf(expf(-a.a_ph * dn), a.k2);
    const float wl = 1.f - wp - wn;
    float dI = 0.f, A[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float L = wl * P[c] + wp * Pp[c] + wn * Pn[c];
      A[c] = wp * G[c] + (1.f - wp) * L;
      const float AI = wl * I[c] + wp * Ip[c] + wn * In[c];
      dI += (I[c] - AI) * (I[c] - AI);
    }
    const float wc = a.lambda * expf(-a.a_ph * dI);
    a.wc[img * plane + pix] = wc;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* Pc = a.P + o3 + c * plane;
      const float pc = P[c];
      float lap = 0.f;
      if (x + 1 < a.w) lap += Pc[pix + 1] - pc;
      if (x > 0) lap += Pc[pix - 1] - pc;
      if (y + 1 < a.h) lap += Pc[pix + a.w] - pc;
      if (y > 0) lap += Pc[pix - a.w] - pc;
      a.R[o3 + c * plane + pix] = wc * A[c] - lap;
      a.O0[o3 + c * plane + pix] = A[c];
      a.O1[o3 + c * plane + pix] = A[c];
    }
  }
}

constexpr int RW = 64, PPT = 12, RH = 4 * PPT;

// Horizontal neighbours through the cross-lane data path (DPP wavefront
// shifts; lane x holds column x of the region): the value of lane x - 1, and
// of lane x + 1 (0 past the wavefront's ends, masked by the callers).
__device__ inline float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ inline float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

// K iterations of the momentum solver on a RW x RH region (K-pixel halo on
// each side, whose values go stale and are not written back).  Wave w holds
// rows PPT w .. PPT w + PPT - 1 of the region in registers, one column per
// lane: horizontal neighbours come from the neighbouring lanes, vertical ones
// from the lane's own rows, except for a strip's first and last rows, whose
// outer neighbours the adjacent waves publish in LDS each iteration (double
// buffered by iteration parity: one barrier per iteration).
__global__ __launch_bounds__(256) void paper_solve_kernel(PaperArgs a, const float* __restrict__ O,
                                                          const float* __restrict__ Oold,
                                                          float* __restrict__ On,
                                                          float* __restrict__ Onold, int K) {
  __shared__ float sx[2][4][2][3][RW];  // [parity][wave][first / last row][channel][column]
  const int tx = threadIdx.x & 63, tg = threadIdx.x >> 6;
  const int TWo = RW - 2 * K, THo = RH - 2 * K;
  const uint3 tile = xcd_tile();
  const int img = tile.z;
  const int gx = tile.x * TWo - K + tx;
  const int gy0 = tile.y * THo - K + tg * PPT;
  const size_t plane = (size_t)a.h * a.w;
  const size_t o3 = (size_t)img * 3 * plane;
  const bool colin = gx >= 0 && gx < a.w;

  float o[PPT][3], oo[PPT][3], r[PPT][3], wc[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int gy = gy0 + k;
    const bool in = colin && gy >= 0 && gy < a.h;
    const size_t p = in ? (size_t)gy * a.w + gx : 0;
    wc[k] = in ? a.wc[(size_t)img * plane + p] : 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t q = o3 + c * plane + p;
      o[k][c] = in ? O[q] : 0.f;
      oo[k][c] = in ? Oold[q] : 0.f;
      r[k][c] = in ? a.R[q] : 0.f;
    }
  }
  // in-image neighbours inside the region (outside the region the value is
  // stale anyway and only feeds the discarded border)
  const bool hx1 = gx + 1 < a.w && tx + 1 < RW, hx0 = gx > 0 && tx > 0;

  for (int it = 0; it < K; ++it) {
    float(*ex)[2][3][RW] = sx[it & 1];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ex[tg][0][c][tx] = o[0][c];
      ex[tg][1][c][tx] = o[PPT - 1][c];
    }
    __syncthreads();
    float up[3], dn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      up[c] = tg > 0 ? ex[tg - 1][1][c][tx] : 0.f;
      dn[c] = tg < 3 ? ex[tg + 1][0][c][tx] : 0.f;
    }
    float no[PPT][3];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int ly = tg * PPT + k, gy = gy0 + k;
      const bool hy1 = gy + 1 < a.h && ly + 1 < RH, hy0 = gy > 0 && ly > 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float cen = o[k][c];
        const float right = from_right(cen), left = from_left(cen);
        const float below = k + 1 < PPT ? o[k + 1][c] : dn[c];
        const float above = k > 0 ? o[k - 1][c] : up[c];
        float lap = 0.f;
        if (hx1) lap += right - cen;
        if (hx0) lap += left - cen;
        if (hy1) lap += below - cen;
        if (hy0) lap += above - cen;
        const float grad = -lap + wc[k] * cen - r[k][c];
        no[k][c] = cen - a.eta * grad + a.kappa * (cen - oo[k][c]);
      }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        oo[k][c] = o[k][c];
        o[k][c] = no[k][c];
      }
  }

  // write back the interior
  if (!colin || tx < K || tx >= RW - K) return;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int ly = tg * PPT + k, gy = gy0 + k;
    if (ly < K || ly >= RH - K || gy < 0 || gy >= a.h) continue;
    const size_t p = (size_t)gy * a.w + gx;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      On[o3 + c * plane + p] = o[k][c];
      Onold[o3 + c * plane + p] = oo[k][c];
    }
  }
}

}  // namespace

hipError_t launch_paper_step(const PaperArgs& a, float* out, int block_iters, hipStream_t s) {
  const size_t total = (size_t)a.n * a.h * a.w;
  if (!total) return hipSuccess;
  if (block_iters < 1 || 2 * block_iters >= RH) return hipErrorInvalidValue;
  size_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  paper_reference_kernel<<<(unsigned)g, 256, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // ping-pong: (O0, O1) -> (O2, O3) -> (O0, O1) ...; the last pass writes `out`
  float* cur[2] = {a.O0, a.O1};
  float* nxt[2] = {a.O2, a.O3};
  int left = a.iters;
  if (left == 0) return hipMemcpyAsync(out, a.O0, total * 3 * sizeof(float),
                                       hipMemcpyDeviceToDevice, s);
  while (left > 0) {
    const int K = left < block_iters ? left : block_iters;
    left -= K;
    float* dst = left == 0 ? out : nxt[0];
    dim3 grid(cdiv(a.w, RW - 2 * K), cdiv(a.h, RH - 2 * K), a.n);
    paper_solve_kernel<<<grid, 256, 0, s>>>(a, cur[0], cur[1], dst, nxt[1], K);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    float* t0 = cur[0];
    float* t1 = cur[1];
    cur[0] = nxt[0];
    cur[1] = nxt[1];
    nxt[0] = t0;
    nxt[1] = t1;
  }
  return hipSuccess;
}

}  // namespace tc
