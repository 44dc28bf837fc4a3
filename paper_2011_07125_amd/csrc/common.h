// Device-side helpers shared by the HIP kernels of libferminet (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fn {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), both rounded to
// nearest even by the hardware conversion (v_cvt_pk_bf16_f32 on gfx950)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
// the same split for two values at once, packed (element 0 in the low half):
// one v_cvt_pk_bf16_f32 per part
__device__ inline void split_bf16x2(float x0, float x1, uint32_t* hi, uint32_t* lo) {
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){x0, x1}, bf16x2));
  const float h0 = __builtin_bit_cast(float, h << 16), h1 = __builtin_bit_cast(float, h & 0xffff0000u);
  *hi = h;
  *lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){x0 - h0, x1 - h1}, bf16x2));
}
// x = h + m + l in three bfloat16 parts for two values at once (packed):
// h = bf16(x), m = bf16(x - h), l = bf16(x - h - m); the differences are
// exact in float32, so the three parts carry every significand bit of x
// (l rounds away at most a bit below 2^-24 |x|)
__device__ inline void split3_bf16x2(float x0, float x1, uint32_t* h, uint32_t* m, uint32_t* l) {
  const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){x0, x1}, bf16x2));
  const float r0 = x0 - __builtin_bit_cast(float, hb << 16), r1 = x1 - __builtin_bit_cast(float, hb & 0xffff0000u);
  const uint32_t mb = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){r0, r1}, bf16x2));
  const float s0 = r0 - __builtin_bit_cast(float, mb << 16), s1 = r1 - __builtin_bit_cast(float, mb & 0xffff0000u);
  *h = hb;
  *m = mb;
  *l = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){s0, s1}, bf16x2));
}
__device__ inline void split_bf16(float x, uint16_t* h, uint16_t* l) {
  const __bf16 hb = (__bf16)x;
  const __bf16 lb = (__bf16)(x - (float)hb);
  *h = __builtin_bit_cast(uint16_t, hb);
  *l = __builtin_bit_cast(uint16_t, lb);
}

// tanh'(u) = sech^2(u) = 4 e^{-2|u|} / (1 + e^{-2|u|})^2, free of the
// cancellation of 1 - tanh^2(u) once tanh saturates
__device__ inline float sech2f(float u) {
  const float e = expf(-2.0f * fabsf(u));
  const float d = 1.0f + e;
  return 4.0f * e / (d * d);
}

// tanh(u) and sech^2(u) from one expm1: with m = e^{-2|u|} - 1,
//   tanh|u| = -m / (2 + m),  sech^2 u = 4 (1 + m) / (2 + m)^2
// (no cancellation for small |u| or once tanh saturates)
// 1 / d for d in [1, 2] is the hardware reciprocal refined by one Newton
// step (r + r (1 - d r)), which leaves about half an ulp.
__device__ inline void tanh_sech2f(float u, float* th, float* s2) {
  const float m = expm1f(-2.0f * fabsf(u));
  const float d = 2.0f + m;
  float r = __builtin_amdgcn_rcpf(d);
  r = fmaf(r, fmaf(-d, r, 1.0f), r);
  const float t = -m * r;
  *th = u < 0.0f ? -t : t;
  *s2 = 4.0f * (1.0f + m) * (r * r);
}
__device__ inline void tanh_sech2(float u, float* th, float* s2) { tanh_sech2f(u, th, s2); }
__device__ inline void tanh_sech2(double u, double* th, double* s2) {
  const double m = expm1(-2.0 * fabs(u));
  const double d = 2.0 + m;
  const double t = -m / d;
  *th = u < 0.0 ? -t : t;
  *s2 = 4.0 * (1.0 + m) / (d * d);
}

template <class T> __device__ inline T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
template <class T> __device__ inline T wave_max(T v) {
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace fn
