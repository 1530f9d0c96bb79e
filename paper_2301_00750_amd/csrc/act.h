// Device helpers for activation storage: float32 or bfloat16 (stored as the
// upper 16 bits of a float, round-to-nearest-even), blocks of 8 channels.
#pragma once
#include <hip/hip_runtime.h>

namespace tc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;  // storage type of bfloat16 activations

// Orders the LDS accesses of one wave's lanes around it: lanes of a wave that
// exchange data through a region only that wave touches need no workgroup
// barrier (a wave's LDS instructions run in order), only this compiler-level
// ordering.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline float bf2f(bf16 h) { return __uint_as_float((unsigned)h << 16); }

// Load through the global address space (global_load_*).  Pointers picked
// from views or device tables are generic, and generic (flat) loads also
// count against the LDS wait counter: every wait for an LDS read would then
// wait for the prefetch of the next chunk as well.
template <typename T>
__device__ inline T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

// float -> bfloat16 with the hardware conversion (v_cvt_pk_bf16_f32: round to
// nearest even; NaN stays NaN).
__device__ inline unsigned pack2(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(float2v{a, b}, bf16x2));
}

__device__ inline bf16 f2bf(float f) { return (bf16)(pack2(f, 0.f) & 0xffffu); }

__device__ inline void load8(const float* p, float (&v)[8]) {
  const f4 a = reinterpret_cast<const f4*>(p)[0], b = reinterpret_cast<const f4*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ inline void load8(const bf16* p, float (&v)[8]) {
  const u4 x = *reinterpret_cast<const u4*>(p);
  v[0] = __uint_as_float(x.x << 16); v[1] = __uint_as_float(x.x & 0xffff0000u);
  v[2] = __uint_as_float(x.y << 16); v[3] = __uint_as_float(x.y & 0xffff0000u);
  v[4] = __uint_as_float(x.z << 16); v[5] = __uint_as_float(x.z & 0xffff0000u);
  v[6] = __uint_as_float(x.w << 16); v[7] = __uint_as_float(x.w & 0xffff0000u);
}

// load8 from global memory (see ldg)
__device__ inline void load8g(const float* p, float (&v)[8]) {
  const f4 a = ldg(reinterpret_cast<const f4*>(p)), b = ldg(reinterpret_cast<const f4*>(p) + 1);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ inline void load8g(const bf16* p, float (&v)[8]) {
  const u4 x = ldg(reinterpret_cast<const u4*>(p));
  v[0] = __uint_as_float(x.x << 16); v[1] = __uint_as_float(x.x & 0xffff0000u);
  v[2] = __uint_as_float(x.y << 16); v[3] = __uint_as_float(x.y & 0xffff0000u);
  v[4] = __uint_as_float(x.z << 16); v[5] = __uint_as_float(x.z & 0xffff0000u);
  v[6] = __uint_as_float(x.w << 16); v[7] = __uint_as_float(x.w & 0xffff0000u);
}

__device__ inline void store8(float* p, const float (&v)[8]) {
  reinterpret_cast<f4*>(p)[0] = f4{v[0], v[1], v[2], v[3]};
  reinterpret_cast<f4*>(p)[1] = f4{v[4], v[5], v[6], v[7]};
}

__device__ inline void store8(bf16* p, const float (&v)[8]) {
  *reinterpret_cast<u4*>(p) =
      u4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
}

__device__ inline void store1(float* p, float v) { *p = v; }
__device__ inline void store1(bf16* p, float v) { *p = f2bf(v); }

// float16 activations (the pyramid features of the BF16 and FP8 forms: the
// cost volume's inputs), round to nearest even.
typedef _Float16 f16;
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ inline unsigned pack2h(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(float2v{a, b}, h2));
}

__device__ inline void unpack8h(const u4& x, float (&v)[8]) {
  const unsigned wd[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const h2 p = __builtin_bit_cast(h2, wd[k]);
    v[2 * k] = (float)p.x;
    v[2 * k + 1] = (float)p.y;
  }
}

__device__ inline void load8(const f16* p, float (&v)[8]) {
  unpack8h(*reinterpret_cast<const u4*>(p), v);
}

__device__ inline void load8g(const f16* p, float (&v)[8]) {
  unpack8h(ldg(reinterpret_cast<const u4*>(p)), v);
}

__device__ inline void store8(f16* p, const float (&v)[8]) {
  *reinterpret_cast<u4*>(p) =
      u4{pack2h(v[0], v[1]), pack2h(v[2], v[3]), pack2h(v[4], v[5]), pack2h(v[6], v[7])};
}

__device__ inline void store1(f16* p, float v) { *p = (f16)v; }

// 8 float16 values (one 16-byte word) -> 8 bfloat16 (round to nearest even).
__device__ inline u4 h8_to_bf8(const u4& x) {
  float v[8];
  unpack8h(x, v);
  return u4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
}

}  // namespace tc

namespace tc {

typedef unsigned int u2v __attribute__((ext_vector_type(2)));

// Largest finite value of FP8 E4M3 (OCP "fn" variant used by gfx950).
constexpr float kFp8Max = 448.f;

// 8 floats -> 8 FP8 E4M3 (round to nearest even, saturated to +-448), after
// multiplying by `inv_scale`.
__device__ inline u2v pack8_fp8(const float (&v)[8], float inv_scale) {
  float s[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) s[i] = fminf(fmaxf(v[i] * inv_scale, -kFp8Max), kFp8Max);
  int lo = __builtin_amdgcn_cvt_pk_fp8_f32(s[0], s[1], 0, false);
  lo = __builtin_amdgcn_cvt_pk_fp8_f32(s[2], s[3], lo, true);
  int hi = __builtin_amdgcn_cvt_pk_fp8_f32(s[4], s[5], 0, false);
  hi = __builtin_amdgcn_cvt_pk_fp8_f32(s[6], s[7], hi, true);
  return u2v{(unsigned)lo, (unsigned)hi};
}

// One 16-byte word of 8 bfloat16 (f16 = false) or float16 values to 8 FP8
// E4M3 bytes, each value divided by s, by gfx950's scaled packed conversions
// (two values per instruction).  The instruction applies only the exponent
// of its scale, so s must be a power of two; a quotient beyond 448 becomes
// NaN, so s must bound the values.  The word's components are copied to
// scalars before the bit casts (a bit cast of a vector element can read
// element 0).
__device__ inline u2v word_to_fp8_pow2(u4 w, bool f16, float s) {
  typedef short s2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  const unsigned c[4] = {w.x, w.y, w.z, w.w};
  s2 lo = {0, 0}, hi = {0, 0};
  if (f16) {
    lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(lo, __builtin_bit_cast(h2, c[0]), s, false);
    lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(lo, __builtin_bit_cast(h2, c[1]), s, true);
    hi = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(hi, __builtin_bit_cast(h2, c[2]), s, false);
    hi = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(hi, __builtin_bit_cast(h2, c[3]), s, true);
  } else {
    lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16(lo, __builtin_bit_cast(b2, c[0]), s, false);
    lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16(lo, __builtin_bit_cast(b2, c[1]), s, true);
    hi = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16(hi, __builtin_bit_cast(b2, c[2]), s, false);
    hi = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16(hi, __builtin_bit_cast(b2, c[3]), s, true);
  }
  return u2v{__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)};
}

// The power of two at or above q > 0 (q normal)
__device__ inline float pow2_ceil(float q) {
  const unsigned b = __builtin_bit_cast(unsigned, q);
  return (b & 0x007fffffu) ? __builtin_bit_cast(float, (b & 0x7f800000u) + 0x00800000u) : q;
}

// Each image's absolute maximum is spread over kAmaxSub sub-slots, each on
// its own 128-byte line, so that the workgroups of a kernel do not all hit
// one address; a consumer takes the maximum of the sub-slots.
constexpr int kAmaxSub = 64;
constexpr int kAmaxStride = 32;  // unsigned words between sub-slots
constexpr int kAmaxWords = kAmaxSub * kAmaxStride;  // per image

// Workgroup-wide maximum folded into one of the image's sub-slots with one
// atomic (values are >= 0, so their float bit patterns order like unsigned
// integers; the maximum is independent of arrival order).  Every thread of
// the workgroup (blockDim.x <= 1024) must call this.
__device__ inline void record_amax(unsigned* slots, float v) {
  __shared__ float red[16];
  if (!slots) return;
  v = fabsf(v);
  if (!(v <= 3.0e38f)) v = 3.0e38f;  // NaN / inf saturate
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < nw; ++i) v = fmaxf(v, red[i]);
    const unsigned sub = (blockIdx.x * 7u + blockIdx.y * 13u + blockIdx.z * 29u) % kAmaxSub;
    atomicMax(slots + sub * kAmaxStride, __float_as_uint(v));
  }
}

// Maximum over an image's sub-slots; every lane of the wave must call this.
__device__ inline float read_amax(const unsigned* slots) {
  if (!slots) return 0.f;
  float v = __uint_as_float(slots[(threadIdx.x & (kAmaxSub - 1)) * kAmaxStride]);
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

}  // namespace tc
