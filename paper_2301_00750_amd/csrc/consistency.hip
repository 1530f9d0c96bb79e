// Fused consistency step: backward warp of O_{t-1}, forward-backward
// visibility test, and the alpha-weighted blend with P_t, in one pass.
// Paper Sec. 3.1 (Eq. 4: G_t = warp(O_{t-1}); Eq. 5: blend with the global
// share clamped by the interactive strength) and Sec. 5 (non-occlusion mask
// of Eq. 9 as a forward-backward consistency test).
//
// Bytes per pixel: P 12 + flow_bw 8 + O_{t-1} 12 + flow_fw 8 (gathered near
// the pixel, so read about once) + out 12 = 52 (+1 with the mask).
#include "tc_internal.h"

namespace tc {
namespace {

// Bilinear taps of the point x + f along one axis of length n: integer part
// taken from the flow alone so that the fraction is exact whatever x is.
struct Taps {
  int i0, i1;
  float a;  // weight of i1
};

__device__ inline Taps axis_taps(int x, float f, int n) {
  const float ff = floorf(f);
  Taps t;
  t.a = f - ff;
  const float s = fminf(fmaxf((float)x + ff, -2.f), (float)n + 1.f);
  const int i = (int)s;
  t.i0 = min(max(i, 0), n - 1);
  t.i1 = min(max(i + 1, 0), n - 1);
  return t;
}

// Forward-backward test at pixel (x, y) of one image: the backward flow's
// target must lie in the image and the forward flow sampled there (bilinear)
// must cancel it up to 0.01 (|f_b|^2 + |f~_f|^2) + 0.5.  Returns the taps of
// the target for the warp.
struct Vis {
  bool vis;
  float w00, w01, w10, w11;
  size_t o00, o01, o10, o11;
};

__device__ inline Vis visibility(const float* __restrict__ ff, const float* __restrict__ fb,
                                 size_t plane, size_t pix, int x, int y, int w, int h) {
  const float bx = fb[pix], by = fb[plane + pix];
  // 0 <= x + bx <= w - 1, evaluated exactly in float
  const bool inside = bx >= -(float)x && bx <= (float)(w - 1 - x) && by >= -(float)y &&
                      by <= (float)(h - 1 - y);
  const Taps tx = axis_taps(x, bx, w), ty = axis_taps(y, by, h);
  Vis v;
  v.w00 = (1.f - tx.a) * (1.f - ty.a);
  v.w01 = tx.a * (1.f - ty.a);
  v.w10 = (1.f - tx.a) * ty.a;
  v.w11 = tx.a * ty.a;
  v.o00 = (size_t)ty.i0 * w + tx.i0;
  v.o01 = (size_t)ty.i0 * w + tx.i1;
  v.o10 = (size_t)ty.i1 * w + tx.i0;
  v.o11 = (size_t)ty.i1 * w + tx.i1;
  const float fx = v.w00 * ff[v.o00] + v.w01 * ff[v.o01] + v.w10 * ff[v.o10] + v.w11 * ff[v.o11];
  const float fy = v.w00 * ff[plane + v.o00] + v.w01 * ff[plane + v.o01] +
                   v.w10 * ff[plane + v.o10] + v.w11 * ff[plane + v.o11];
  const float sx = bx + fx, sy = by + fy;
  const float lhs = sx * sx + sy * sy;
  const float rhs = 0.01f * (bx * bx + by * by + fx * fx + fy * fy) + 0.5f;
  v.vis = inside && lhs <= rhs;
  return v;
}

// Number of pixels of each image that pass the test (one atomic per
// workgroup and image; integer, so the count is exact).
__global__ __launch_bounds__(256) void agreement_kernel(const float* __restrict__ ffw,
                                                        const float* __restrict__ fbw, int h,
                                                        int w, unsigned* __restrict__ counts) {
  __shared__ unsigned red[4];
  const size_t plane = (size_t)h * w;
  const int img = blockIdx.y;
  unsigned c = 0;
  for (size_t pix = blockIdx.x * (size_t)blockDim.x + threadIdx.x; pix < plane;
       pix += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(pix / w), x = (int)(pix - (size_t)y * w);
    c += visibility(ffw + (size_t)img * 2 * plane, fbw + (size_t)img * 2 * plane, plane, pix, x,
                    y, w, h).vis;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(counts + img, red[0] + red[1] + red[2] + red[3]);
}

__global__ __launch_bounds__(256) void consistency_kernel(
    const float* P, const float* __restrict__ Oprev, const float* __restrict__ ffw,
    const float* __restrict__ fbw, float alpha, int n, int h, int w, float* out,
    unsigned char* __restrict__ mask) {
  // grid: x over 256-pixel pieces of a row, y = row, z = image (no index
  // division per pixel)
  const size_t plane = (size_t)h * w;
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  const size_t img = blockIdx.z;
  if (x < w) {
    const size_t pix = (size_t)y * w + x, i = img * plane + pix;
    const Vis v = visibility(ffw + img * 2 * plane, fbw + img * 2 * plane, plane, pix, x, y, w, h);
    const bool vis = v.vis;
    const float w00 = v.w00, w01 = v.w01, w10 = v.w10, w11 = v.w11;
    const size_t o00 = v.o00, o01 = v.o01, o10 = v.o10, o11 = v.o11;

    const float* Pi = P + img * 3 * plane;
    const float* Oi = Oprev + img * 3 * plane;
    float* oi = out + img * 3 * plane;
    float res[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* O = Oi + c * plane;
      const float p = Pi[c * plane + pix];
      if (vis) {
        const float g = w00 * O[o00] + w01 * O[o01] + w10 * O[o10] + w11 * O[o11];
        res[c] = (1.f - alpha) * p + alpha * g;
      } else {
        res[c] = p;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) oi[c * plane + pix] = res[c];
    if (mask) mask[i] = vis ? 1 : 0;
  }
}

}  // namespace

hipError_t launch_agreement(const float* ffw, const float* fbw, int n, int h, int w,
                            unsigned* counts, hipStream_t s) {
  const size_t plane = (size_t)h * w;
  if (!n || !plane) return hipSuccess;
  hipError_t e = launch_zero_u32(counts, (size_t)n, s);
  if (e != hipSuccess) return e;
  size_t g = (plane + 255) / 256;
  if (g > 1024) g = 1024;
  agreement_kernel<<<dim3((unsigned)g, (unsigned)n), 256, 0, s>>>(ffw, fbw, h, w, counts);
  return hipGetLastError();
}

hipError_t launch_consistency(const float* P, const float* Oprev, const float* ffw,
                              const float* fbw, float alpha, int n, int h, int w, float* out,
                              unsigned char* mask, hipStream_t s) {
  const size_t total = (size_t)n * h * w;
  if (!total) return hipSuccess;
  consistency_kernel<<<dim3(cdiv(w, 256), h, n), 256, 0, s>>>(P, Oprev, ffw, fbw, alpha, n, h, w,
                                                              out, mask);
  return hipGetLastError();
}

}  // namespace tc
