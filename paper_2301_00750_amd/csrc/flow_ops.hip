// Bandwidth-bound steps of the flow network: frame staging, flow upsampling,
// the fused feature warp + cost volume, and the final upsample-and-crop.
#include <type_traits>

#include "act.h"
#include "tc_internal.h"

namespace tc {
namespace {

// ---------------------------------------------------------------- staging

// T = float: blocks of 4 channels (RGB, 0); T = bf16: blocks of 8 (RGB, 0 x 5).
template <typename T>
__global__ __launch_bounds__(256) void stage_kernel(const float* __restrict__ frames, int n, int h,
                                                    int w, T* __restrict__ out, int hp, int wp,
                                                    unsigned* aout) {
  // grid: x over 256-pixel pieces of a row, y = row, z = image (no index
  // division per pixel)
  const int img = blockIdx.z, y = blockIdx.y;
  const int x = blockIdx.x * 256 + threadIdx.x;
  const size_t per = (size_t)hp * wp;
  float mx = 0.f;
  if (x < wp) {
    const size_t i = (size_t)y * wp + x;
    const int sy = y < h ? y : h - 1, sx = x < w ? x : w - 1;
    const size_t plane = (size_t)h * w;
    const float* f = frames + (size_t)img * 3 * plane + (size_t)sy * w + sx;
    const float r = f[0], g = f[plane], b = f[2 * plane];
    mx = fmaxf(mx, fmaxf(fabsf(r), fmaxf(fabsf(g), fabsf(b))));
    const size_t o = (size_t)img * per + i;
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<f4*>(out + o * 4) = f4{r, g, b, 0.f};
    } else {
      const float v[8] = {r, g, b, 0.f, 0.f, 0.f, 0.f, 0.f};
      store8(out + o * 8, v);
    }
  }
  if (aout) record_amax(aout + (size_t)img * kAmaxWords, mx);
}

__global__ void write_table_kernel(PtrTable t, int n, const void** dst) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = t.p[threadIdx.x];
}

__global__ __launch_bounds__(256) void zero_u32_kernel(unsigned* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------- up2

// Source coordinate of output index i for upsampling by a power of two s
// with half-pixel centres: (i + 1/2) / s - 1/2 clamped to [0, n - 1]; exact
// in float (inv_s = 1 / s).
__device__ inline void up_taps(int i, int n, float inv_s, int& i0, int& i1, float& f) {
  float src = fmaxf((i + 0.5f) * inv_s - 0.5f, 0.f);
  i0 = min((int)src, n - 1);
  f = src - (float)i0;
  if (i0 >= n - 1) f = 0.f;
  i1 = min(i0 + 1, n - 1);
}

__device__ inline void up2_taps(int i, int n, int& i0, int& i1, float& f) {
  up_taps(i, n, 0.5f, i0, i1, f);
}

__global__ __launch_bounds__(256) void up2x2_kernel(const float* __restrict__ flow, int n, int h,
                                                    int w, float* __restrict__ U) {
  const int H = 2 * h, W = 2 * w;
  const size_t total = (size_t)n * H * W;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % W);
    const int y = (int)((i / W) % H);
    const int img = (int)(i / ((size_t)W * H));
    int y0, y1, x0, x1;
    float fy, fx;
    up2_taps(y, h, y0, y1, fy);
    up2_taps(x, w, x0, x1, fx);
    const float2* f = reinterpret_cast<const float2*>(flow) + (size_t)img * h * w;
    const float2 a = f[y0 * w + x0], b = f[y0 * w + x1], c = f[y1 * w + x0], d = f[y1 * w + x1];
    float2 r;
    r.x = 2.f * ((1.f - fy) * ((1.f - fx) * a.x + fx * b.x) + fy * ((1.f - fx) * c.x + fx * d.x));
    r.y = 2.f * ((1.f - fy) * ((1.f - fx) * a.y + fx * b.y) + fy * ((1.f - fx) * c.y + fx * d.y));
    reinterpret_cast<float2*>(U)[i] = r;
  }
}

__global__ __launch_bounds__(256) void final_flow_kernel(const float* __restrict__ flowf, int n,
                                                         int hf, int wf, int scale,
                                                         float* __restrict__ out_a,
                                                         float* __restrict__ out_b, int nsplit,
                                                         int H, int W, float* const* out_tab) {
  // grid: x over 256-pixel pieces of a row, y = row, z = image
  const float sc = (float)scale, inv_s = 1.f / (float)scale;
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, img = blockIdx.z;
  if (x < W) {
    int y0, y1, x0, x1;
    float fy, fx;
    up_taps(y, hf, inv_s, y0, y1, fy);
    up_taps(x, wf, inv_s, x0, x1, fx);
    const float2* f = reinterpret_cast<const float2*>(flowf) + (size_t)img * hf * wf;
    const float2 a = f[y0 * wf + x0], b = f[y0 * wf + x1], c = f[y1 * wf + x0], d = f[y1 * wf + x1];
    const float rx = sc * ((1.f - fy) * ((1.f - fx) * a.x + fx * b.x) + fy * ((1.f - fx) * c.x + fx * d.x));
    const float ry = sc * ((1.f - fy) * ((1.f - fx) * a.y + fx * b.y) + fy * ((1.f - fx) * c.y + fx * d.y));
    float* o = out_tab ? out_tab[img]
               : img < nsplit ? out_a + (size_t)img * 2 * H * W
                              : out_b + (size_t)(img - nsplit) * 2 * H * W;
    o[(size_t)y * W + x] = rx;
    o[(size_t)H * W + (size_t)y * W + x] = ry;
  }
}

// Half-size frames: the mean of each 2x2 pixel block of every plane; a block
// that runs past the last row or column repeats it.
__global__ __launch_bounds__(256) void half_frames_kernel(const float* __restrict__ in, int planes,
                                                          int h, int w, int h2, int w2,
                                                          float* __restrict__ out) {
  const size_t total = (size_t)planes * h2 * w2;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % w2);
    const int y = (int)((i / w2) % h2);
    const size_t p = i / ((size_t)w2 * h2);
    const float* src = in + p * h * w;
    const int y0 = 2 * y, y1 = min(2 * y + 1, h - 1), x0 = 2 * x, x1 = min(2 * x + 1, w - 1);
    out[i] = 0.25f * ((src[(size_t)y0 * w + x0] + src[(size_t)y0 * w + x1]) +
                      (src[(size_t)y1 * w + x0] + src[(size_t)y1 * w + x1]));
  }
}

// Flow (n x 2 x h2 x w2) to n x 2 x H x W: bilinear, half-pixel centres,
// times 2.
__global__ __launch_bounds__(256) void flow_up2_planes_kernel(const float* __restrict__ in, int n,
                                                              int h2, int w2, int H, int W,
                                                              float* __restrict__ out) {
  const size_t total = (size_t)n * H * W;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % W);
    const int y = (int)((i / W) % H);
    const size_t img = i / ((size_t)W * H);
    int y0, y1, x0, x1;
    float fy, fx;
    up2_taps(y, h2, y0, y1, fy);
    up2_taps(x, w2, x0, x1, fx);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float* f = in + (img * 2 + c) * h2 * w2;
      const float a = f[y0 * w2 + x0], b = f[y0 * w2 + x1], cc = f[y1 * w2 + x0],
                  d = f[y1 * w2 + x1];
      out[(img * 2 + c) * H * W + (size_t)y * W + x] =
          2.f * ((1.f - fy) * ((1.f - fx) * a + fx * b) + fy * ((1.f - fx) * cc + fx * d));
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void flow_to_block_kernel(const float* __restrict__ flow, int n,
                                                            int hw, T* __restrict__ out, int cbt,
                                                            int cb) {
  const size_t total = (size_t)n * hw;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t img = i / hw, p = i - img * hw;
    const float2 f = reinterpret_cast<const float2*>(flow)[i];
    const float v[8] = {f.x, f.y, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    store8(out + ((img * cbt + cb) * hw + p) * 8, v);
  }
}

// ---------------------------------------------------------------- warp + cost volume
//
// A workgroup owns a TY x TX tile of pixels (one per thread).  The bilinear
// taps of the tile plus a halo of R pixels (which taps lie inside the image,
// and the fractional offsets) are computed once; then per chunk of 8 channels
// it gathers the warped second-image features into LDS (zero outside), and
// every thread accumulates its (2R+1)^2 correlations from LDS.  Layout of the LDS tile:
// [2 float4 planes][halo positions][4] so that neighbouring lanes read
// neighbouring 16-byte words.

constexpr int CV_TY = 8, CV_TX = 32;

template <typename T>
__device__ inline const T* vbase(const View& v, int img, size_t img_elems) {
  if (v.tab) return reinterpret_cast<const T*>(v.tab[img]);
  return img < v.nsplit ? reinterpret_cast<const T*>(v.a) + (size_t)img * img_elems
                        : reinterpret_cast<const T*>(v.b) + (size_t)(img - v.nsplit) * img_elems;
}

// T = storage type of the features (float, bfloat16 or float16), TZ = of Z.
// Float16 features: the warped F2 tile is rounded to float16 in LDS (one
// 16-byte word per position) and each displacement's 8-channel product is
// four v_dot2_f32_f16 (float16 products, float32 sums).
template <int R, typename T, typename TZ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void warp_cv_kernel(CvArgs a) {
  constexpr int D = 2 * R + 1, NCV = D * D;
  constexpr int HY = CV_TY + 2 * R, HX = CV_TX + 2 * R, NPOS = HY * HX;
  constexpr bool H = std::is_same<T, f16>::value;
  __shared__ f4 s2[2][NPOS];
  u4* s2h = reinterpret_cast<u4*>(&s2[0][0]);  // float16 tile (H)
  __shared__ int2 s_tap[NPOS];     // (pixel index of the top-left tap, validity bits of the 4 taps)
  __shared__ float2 s_frac[NPOS];  // (ax, ay)

  const int tid = threadIdx.x;
  const int lx = tid % CV_TX, ly = tid / CV_TX;
  const int tx0 = blockIdx.x * CV_TX, ty0 = blockIdx.y * CV_TY;
  const int img = blockIdx.z / a.splits, split = blockIdx.z - img * a.splits;
  const int x = tx0 + lx, y = ty0 + ly;
  const bool valid = x < a.w && y < a.h;
  const int h = a.h, w = a.w;
  const size_t plane = (size_t)h * w * 8;
  const int cb_begin = split * a.cps;
  const int cb_end = min(a.C / 8, cb_begin + a.cps);
  const T* f1 = vbase<T>(a.f1, img, plane * a.f1.cbt);
  const T* f2 = vbase<T>(a.f2, img, plane * a.f2.cbt);
  const float2* U = a.U ? reinterpret_cast<const float2*>(a.U) + (size_t)img * h * w : nullptr;

  float acc[NCV];
#pragma unroll
  for (int k = 0; k < NCV; ++k) acc[k] = 0.f;

  // The bilinear taps of every halo position (top-left pixel index, which of
  // the 4 taps lie inside the image, fractional offsets) do not depend on the
  // channel chunk: computed once, kept in LDS.
  for (int p = tid; p < NPOS; p += 256) {
    const int py = p / HX, px = p - py * HX;
    const int Y = ty0 - R + py, X = tx0 - R + px;
    int base = 0, mask = 0;
    float ax = 0.f, ay = 0.f;
    if (Y >= 0 && Y < h && X >= 0 && X < w) {
      if (!U) {
        base = Y * w + X;
        mask = 1;
      } else {
        const float2v u = ldg(reinterpret_cast<const float2v*>(U + (size_t)Y * w + X));
        const float fx = floorf(u.x), fy = floorf(u.y);
        ax = u.x - fx;
        ay = u.y - fy;
        const int x0 = X + (int)fx, y0 = Y + (int)fy;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int xi = x0 + (t & 1), yi = y0 + (t >> 1);
          if (xi >= 0 && xi < w && yi >= 0 && yi < h) mask |= 1 << t;
        }
        if (mask) base = y0 * w + x0;  // -1 <= x0 < w, -1 <= y0 < h here
      }
    }
    s_tap[p] = int2{base, mask};
    s_frac[p] = float2{ax, ay};
  }
  __syncthreads();

  // With FP32 activations the tap loads are unconditional: an index clamped
  // into the image plane, the value of a tap outside the image replaced by
  // zero after the load, so the 4 taps' loads are in flight together (loads
  // inside per-tap branches each wait for their data at the branch join).
  // With BF16 activations the branches measured faster.
  const int last_px = h * w - 1;
  for (int cb = cb_begin; cb < cb_end; ++cb) {
    const T* f2c = f2 + (size_t)cb * plane;
    // BF16: this pixel's F1 chunk (one 16-byte word) is loaded before the
    // gather so that its latency overlaps the gather and the barrier (with
    // FP32 activations the 8 registers this takes spill)
    u4 f1w = u4{0, 0, 0, 0};
    if constexpr (sizeof(T) == 2)
      f1w = ldg(reinterpret_cast<const u4*>(f1 + (size_t)cb * plane +
                                            ((size_t)(valid ? y : 0) * w + (valid ? x : 0)) * 8));
    for (int p = tid; p < NPOS; p += 256) {
      const int2 tp = s_tap[p];
      if constexpr (H) {
        u4 word = u4{0u, 0u, 0u, 0u};
        if (!U) {
          if (tp.y) word = ldg(reinterpret_cast<const u4*>(f2c + (size_t)tp.x * 8));
        } else {
          const float2 fr = s_frac[p];
          float acc8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            if ((tp.y >> t) & 1) {
              const float wt = ((t & 1) ? fr.x : 1.f - fr.x) * ((t >> 1) ? fr.y : 1.f - fr.y);
              float v[8];
              load8g(f2c + ((size_t)tp.x + (t & 1) + (t >> 1) * (size_t)w) * 8, v);
#pragma unroll
              for (int e = 0; e < 8; ++e) acc8[e] = fmaf(wt, v[e], acc8[e]);
            }
          }
          word = u4{pack2h(acc8[0], acc8[1]), pack2h(acc8[2], acc8[3]),
                    pack2h(acc8[4], acc8[5]), pack2h(acc8[6], acc8[7])};
        }
        s2h[p] = word;
        continue;
      }
      f4 lo = f4{0.f, 0.f, 0.f, 0.f}, hi = lo;
      if (!U) {
        if (sizeof(T) == 4 || tp.y) {
          float v[8];
          load8g(f2c + (size_t)tp.x * 8, v);  // tp.x = 0 when the position is outside
          if (tp.y) {
            lo = f4{v[0], v[1], v[2], v[3]};
            hi = f4{v[4], v[5], v[6], v[7]};
          }
        }
      } else if constexpr (sizeof(T) == 2) {
        const float2 fr = s_frac[p];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if ((tp.y >> t) & 1) {
            const float wt = ((t & 1) ? fr.x : 1.f - fr.x) * ((t >> 1) ? fr.y : 1.f - fr.y);
            float v[8];
            load8g(f2c + ((size_t)tp.x + (t & 1) + (t >> 1) * (size_t)w) * 8, v);
            lo += wt * f4{v[0], v[1], v[2], v[3]};
            hi += wt * f4{v[4], v[5], v[6], v[7]};
          }
        }
      } else {
        const float2 fr = s_frac[p];
        float v[4][8];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          load8g(f2c + (size_t)min(max(tp.x + (t & 1) + (t >> 1) * w, 0), last_px) * 8, v[t]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bool in = (tp.y >> t) & 1;
          const float wt = ((t & 1) ? fr.x : 1.f - fr.x) * ((t >> 1) ? fr.y : 1.f - fr.y);
#pragma unroll
          for (int e = 0; e < 8; ++e) v[t][e] = in ? v[t][e] : 0.f;
          lo += wt * f4{v[t][0], v[t][1], v[t][2], v[t][3]};
          hi += wt * f4{v[t][4], v[t][5], v[t][6], v[t][7]};
        }
      }
      s2[0][p] = lo;
      s2[1][p] = hi;
    }
    __syncthreads();
    if (H && valid) {
      // (vector components are copied to plain arrays before the bit casts:
      // hipcc's __builtin_bit_cast of an ext_vector component reads the
      // vector's first component)
      const unsigned aw[4] = {f1w.x, f1w.y, f1w.z, f1w.w};
      h2 av[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) av[k] = __builtin_bit_cast(h2, aw[k]);
#pragma unroll
      for (int dy = 0; dy < D; ++dy)
#pragma unroll
        for (int dx = 0; dx < D; ++dx) {
          const u4 b = s2h[(ly + dy) * HX + lx + dx];
          const unsigned bw[4] = {b.x, b.y, b.z, b.w};
          float sacc = acc[dy * D + dx];
#pragma unroll
          for (int k = 0; k < 4; ++k)
            sacc = __builtin_amdgcn_fdot2(av[k], __builtin_bit_cast(h2, bw[k]), sacc, false);
          acc[dy * D + dx] = sacc;
        }
    } else if (valid) {
      float v1[8];
      if constexpr (sizeof(T) == 2) {
        const unsigned wd[4] = {f1w.x, f1w.y, f1w.z, f1w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          v1[2 * k] = __uint_as_float(wd[k] << 16);
          v1[2 * k + 1] = __uint_as_float(wd[k] & 0xffff0000u);
        }
      } else {
        load8g(f1 + (size_t)cb * plane + ((size_t)y * w + x) * 8, v1);
      }
      const f4 a0 = f4{v1[0], v1[1], v1[2], v1[3]}, a1 = f4{v1[4], v1[5], v1[6], v1[7]};
#pragma unroll
      for (int dy = 0; dy < D; ++dy)
#pragma unroll
        for (int dx = 0; dx < D; ++dx) {
          const int p = (ly + dy) * HX + lx + dx;
          const f4 b0 = s2[0][p], b1 = s2[1][p];
          float s = acc[dy * D + dx];
          s = fmaf(a0.x, b0.x, s);
          s = fmaf(a0.y, b0.y, s);
          s = fmaf(a0.z, b0.z, s);
          s = fmaf(a0.w, b0.w, s);
          s = fmaf(a1.x, b1.x, s);
          s = fmaf(a1.y, b1.y, s);
          s = fmaf(a1.z, b1.z, s);
          s = fmaf(a1.w, b1.w, s);
          acc[dy * D + dx] = s;
        }
    }
    __syncthreads();
  }
  if (a.splits > 1) {  // uniform over the grid
    if (!valid) return;
    float* pp = a.partial + ((size_t)(split * a.n + img) * NCV) * h * w + (size_t)y * w + x;
#pragma unroll
    for (int k = 0; k < NCV; ++k) pp[(size_t)k * h * w] = acc[k];
    return;
  }

  // Z: blocks of 8 channels, [cv 0..NCV-1 | U_x | U_y | 0 ...]
  float mx = 0.f;
  if (valid) {
    const float invC = 1.f / (float)a.C;
    float ux = 0.f, uy = 0.f;
    if (U) {
      const float2 u = U[(size_t)y * w + x];
      ux = u.x;
      uy = u.y;
    }
    constexpr int ZCB = (NCV + 2 + 7) / 8;
    TZ* z = reinterpret_cast<TZ*>(a.Z) + (size_t)img * ZCB * plane + ((size_t)y * w + x) * 8;
#pragma unroll
    for (int b = 0; b < ZCB; ++b) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = b * 8 + e;
        float val = 0.f;
        if (c < NCV) {
          val = acc[c] * invC;
          val = val >= 0.f ? val : a.slope * val;
        } else if (c == NCV) {
          val = ux;
        } else if (c == NCV + 1) {
          val = uy;
        }
        v[e] = val;
        mx = fmaxf(mx, fabsf(val));
      }
      store8(z + (size_t)b * plane, v);
    }
  }
  // every lane of the wave reaches this call (it reduces across the wave)
  if (a.aout) record_amax(a.aout + (size_t)img * kAmaxWords, mx);
}

// Adds the channel splits of the cost volume in split order and writes Z:
// one thread per (pixel, channel of Z), neighbouring threads on neighbouring
// pixels so the partial reads are coalesced.
template <int R, typename T>
__global__ __launch_bounds__(256) void cv_reduce_kernel(CvArgs a) {
  constexpr int D = 2 * R + 1, NCV = D * D, ZCB = (NCV + 2 + 7) / 8;
  const size_t hw = (size_t)a.h * a.w;
  const size_t per = (size_t)ZCB * 8 * hw;
  const int img = blockIdx.y;
  const float invC = 1.f / (float)a.C;
  float mx = 0.f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < per;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t pix = i % hw;
    const int c = (int)(i / hw);
    float val = 0.f;
    if (c < NCV) {
      for (int s = 0; s < a.splits; ++s)
        val += a.partial[((size_t)(s * a.n + img) * NCV + c) * hw + pix];
      val *= invC;
      val = val >= 0.f ? val : a.slope * val;
    } else if (c == NCV || c == NCV + 1) {
      val = a.U ? a.U[((size_t)img * hw + pix) * 2 + (c - NCV)] : 0.f;
    }
    mx = fmaxf(mx, fabsf(val));
    store1(reinterpret_cast<T*>(a.Z) + ((size_t)img * ZCB + (c >> 3)) * hw * 8 + pix * 8 + (c & 7),
           val);
  }
  if (a.aout) record_amax(a.aout + (size_t)img * kAmaxWords, mx);
}

int grid_for(size_t total) {
  size_t g = (total + 255) / 256;
  return (int)(g < 65536 ? g : 65536);
}

}  // namespace

hipError_t launch_stage(const float* frames, int n, int h, int w, float* out, int hp, int wp,
                        int bf16act, unsigned* aout, hipStream_t s) {
  const size_t per = (size_t)hp * wp;
  if (!per || n <= 0) return hipSuccess;
  dim3 grid(cdiv(wp, 256), hp, n);
  if (bf16act)
    stage_kernel<bf16><<<grid, 256, 0, s>>>(frames, n, h, w, reinterpret_cast<bf16*>(out), hp, wp,
                                            aout);
  else
    stage_kernel<float><<<grid, 256, 0, s>>>(frames, n, h, w, out, hp, wp, aout);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  zero_u32_kernel<<<grid_for(n), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_up2x2(const float* flow, int n, int h, int w, float* U, hipStream_t s) {
  const size_t total = (size_t)n * 4 * h * w;
  if (!total) return hipSuccess;
  up2x2_kernel<<<grid_for(total), 256, 0, s>>>(flow, n, h, w, U);
  return hipGetLastError();
}

hipError_t launch_final_flow(const float* flow_f, int n, int hf, int wf, int scale, float* out_a,
                             float* out_b, int nsplit, int H, int W, float* const* out_tab,
                             hipStream_t s) {
  const size_t total = (size_t)n * H * W;
  if (!total) return hipSuccess;
  if (scale < 2 || (scale & (scale - 1)) || (long)hf * scale < H || (long)wf * scale < W)
    return hipErrorInvalidValue;
  final_flow_kernel<<<dim3(cdiv(W, 256), H, n), 256, 0, s>>>(flow_f, n, hf, wf, scale, out_a, out_b, nsplit,
                                                    H, W, out_tab);
  return hipGetLastError();
}

hipError_t launch_half_frames(const float* in, int planes, int h, int w, float* out,
                              hipStream_t s) {
  const int h2 = (h + 1) / 2, w2 = (w + 1) / 2;
  const size_t total = (size_t)planes * h2 * w2;
  if (!total) return hipSuccess;
  half_frames_kernel<<<grid_for(total), 256, 0, s>>>(in, planes, h, w, h2, w2, out);
  return hipGetLastError();
}

hipError_t launch_flow_up2_planes(const float* in, int n, int h2, int w2, int H, int W, float* out,
                                  hipStream_t s) {
  const size_t total = (size_t)n * H * W;
  if (!total) return hipSuccess;
  if (2L * h2 < H || 2L * w2 < W) return hipErrorInvalidValue;
  flow_up2_planes_kernel<<<grid_for(total), 256, 0, s>>>(in, n, h2, w2, H, W, out);
  return hipGetLastError();
}

hipError_t launch_flow_to_block(const float* flow, int n, int hw, void* out, int cbt, int cb,
                                int as_bf16, hipStream_t s) {
  const size_t total = (size_t)n * hw;
  if (!total) return hipSuccess;
  if (as_bf16)
    flow_to_block_kernel<bf16><<<grid_for(total), 256, 0, s>>>(flow, n, hw,
                                                               static_cast<bf16*>(out), cbt, cb);
  else
    flow_to_block_kernel<float><<<grid_for(total), 256, 0, s>>>(flow, n, hw,
                                                                static_cast<float*>(out), cbt, cb);
  return hipGetLastError();
}

hipError_t launch_write_table(const PtrTable& t, int n, const void** dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kTabMax) return hipErrorInvalidValue;
  write_table_kernel<<<1, kTabMax, 0, s>>>(t, n, dst);
  return hipGetLastError();
}

CvPlan plan_cost_volume(int h, int w, int C) {
  // Per-image geometry only (results do not depend on the batch): split the
  // channel chunks when one image has fewer than 128 tiles (below that the
  // grid leaves most CUs idle; above it the split's partial sums and their
  // reduction pass cost more than they save).
  CvPlan p{1, C / 8};
  const long tiles = (long)cdiv(h, CV_TY) * cdiv(w, CV_TX);
  const int nch = C / 8;
  if (tiles < 128 && nch > 1) {
    int splits = (int)((512 + tiles - 1) / tiles);
    if (splits > nch) splits = nch;
    p.cps = cdiv(nch, splits);
    p.splits = cdiv(nch, p.cps);
  }
  return p;
}

size_t cost_volume_partial_bytes(const CvPlan& p, int n, int h, int w) {
  return p.splits > 1 ? (size_t)p.splits * n * 81 * h * w * sizeof(float) : 0;
}

hipError_t launch_warp_cost_volume(const CvArgs& a, hipStream_t s) {
  if (a.radius != 4 || a.C % 8 != 0 || a.zcb != (81 + 2 + 7) / 8) return hipErrorInvalidValue;
  if (a.splits < 1 || a.cps < 1 || (a.splits > 1 && !a.partial)) return hipErrorInvalidValue;
  dim3 grid(cdiv(a.w, CV_TX), cdiv(a.h, CV_TY), a.n * a.splits);
  if (a.bf16act && a.f16feat)
    warp_cv_kernel<4, f16, bf16><<<grid, 256, 0, s>>>(a);
  else if (a.bf16act)
    warp_cv_kernel<4, bf16, bf16><<<grid, 256, 0, s>>>(a);
  else
    warp_cv_kernel<4, float, float><<<grid, 256, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.splits == 1) return e;
  const dim3 g(grid_for((size_t)a.zcb * 8 * a.h * a.w), a.n);
  if (a.bf16act)
    cv_reduce_kernel<4, bf16><<<g, 256, 0, s>>>(a);
  else
    cv_reduce_kernel<4, float><<<g, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace tc
