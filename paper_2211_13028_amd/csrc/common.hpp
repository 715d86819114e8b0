// Internal helpers shared by the HIP kernels and the host library of rtucker.
// gfx950 (CDNA4) only: 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "../../include/rtucker.h"

namespace rt {

constexpr int kWave = 64;

typedef uint16_t bf16_t;  // storage of a bfloat16 value
typedef uint8_t f8_t;     // storage of an OCP E4M3 value

// ---------------------------------------------------------------- widening loads
__device__ __forceinline__ float bf16_to_f32(bf16_t v) {
  return __uint_as_float(static_cast<uint32_t>(v) << 16);
}

// E4M3 (bias 7, 3 fraction bits, 0x7f/0xff NaN) -> binary32, exact.
__device__ __forceinline__ float f8_to_f32(f8_t v) {
  const uint32_t s = (v & 0x80u) << 24;
  const uint32_t e = (v >> 3) & 0xFu;
  const uint32_t m = v & 0x7u;
  if (e == 0xFu && m == 0x7u) return __uint_as_float(0x7fc00000u | s);
  if (e == 0) {
    const float v = static_cast<float>(m) * 0.001953125f;  // subnormal: m * 2^-9
    return s ? -v : v;
  }
  return __uint_as_float(s | ((e + 120u) << 23) | (m << 20));
}

// ---------------------------------------------------------------- global address space
// Pointers that a kernel reads from a job table in memory are generic to the compiler, so
// its accesses through them become FLAT instructions, which count on the LDS counter as
// well: every LDS wait then also waits for the loads in flight.  Casting to the global
// address space gives global loads and stores.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> global_ptr(T* p) {
  return (gptr<T>)(p);
}

// f(integral_constant<int, I>) for I = 0, 1, ... in order
template <class F, int... I>
__device__ __forceinline__ void for_each_index(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}

template <typename T> struct Load;
template <> struct Load<double> { __device__ static double get(const double* p, int64_t i) { return p[i]; } };
template <> struct Load<float> { __device__ static float get(const float* p, int64_t i) { return p[i]; } };
template <> struct Load<bf16_t> { __device__ static float get(const bf16_t* p, int64_t i) { return bf16_to_f32(p[i]); } };
template <> struct Load<f8_t> { __device__ static float get(const f8_t* p, int64_t i) { return f8_to_f32(p[i]); } };

// ---------------------------------------------------------------- rounding (RNE)
// binary64 -> bfloat16 bits, round to nearest even (via the exact binary64 value,
// so no double rounding through binary32).
__device__ __forceinline__ bf16_t f64_to_bf16_bits(double x) {
  uint64_t u = static_cast<uint64_t>(__double_as_longlong(x));
  const uint64_t sign = u >> 63;
  uint64_t a = u & 0x7fffffffffffffffull;
  if (a > 0x7ff0000000000000ull) return static_cast<bf16_t>((sign << 15) | 0x7fc0u);  // NaN
  const int e = static_cast<int>(a >> 52);  // biased binary64 exponent
  // bf16 normal range: biased f32 exponent 1..254 <=> binary64 biased exponent 897..1150
  if (e >= 897) {
    // keep 7 fraction bits out of 52: drop 45 bits with RNE
    const uint64_t lsb = (a >> 45) & 1u;
    a += (1ull << 44) - 1 + lsb;
    uint64_t r = a >> 45;  // exponent(11) | fraction(7), binary64 bias
    int64_t ef = static_cast<int64_t>(r >> 7) - 1023 + 127;
    if (ef >= 255) return static_cast<bf16_t>((sign << 15) | 0x7f80u);  // overflow -> Inf
    return static_cast<bf16_t>((sign << 15) | (static_cast<uint64_t>(ef) << 7) | (r & 0x7fu));
  }
  // subnormal range of bf16 (|x| < 2^-126): quantum 2^-133
  if (e == 0) return static_cast<bf16_t>(sign << 15);
  // value = 1.f * 2^(e-1023); shift so that the integer part counts quanta 2^-133
  const uint64_t mant = (a & 0xfffffffffffffull) | (1ull << 52);
  const int sh = 52 - (e - 1023 + 133);  // number of bits to drop
  if (sh >= 64) return static_cast<bf16_t>(sign << 15);
  uint64_t q = mant >> sh;
  const uint64_t rem = mant & ((1ull << sh) - 1);
  const uint64_t half = 1ull << (sh - 1);
  if (rem > half || (rem == half && (q & 1u))) q += 1;
  return static_cast<bf16_t>((sign << 15) | q);  // q <= 128 -> may become min normal, fine
}

// binary64 -> E4M3 bits, round to nearest even, saturating to +-448; NaN/Inf -> NaN.
__device__ __forceinline__ f8_t f64_to_f8_bits(double x) {
  uint64_t u = static_cast<uint64_t>(__double_as_longlong(x));
  const uint32_t sign = static_cast<uint32_t>(u >> 63) << 7;
  uint64_t a = u & 0x7fffffffffffffffull;
  if (a >= 0x7ff0000000000000ull) return static_cast<f8_t>(sign | 0x7fu);
  const int e = static_cast<int>(a >> 52) - 1023;  // unbiased exponent (a != 0 normal binary64)
  if (a == 0) return static_cast<f8_t>(sign);
  const uint64_t mant = (a & 0xfffffffffffffull) | (1ull << 52);
  // quantum: 2^(e-3) for e >= -6, 2^-9 below
  const int qexp = (e >= -6) ? (e - 3) : -9;
  const int sh = 52 - (e - qexp);  // bits of mant below the quantum
  if (sh >= 64) return static_cast<f8_t>(sign);
  uint64_t q = mant >> sh;
  const uint64_t rem = mant & ((1ull << sh) - 1);
  const uint64_t half = 1ull << (sh - 1);
  if (rem > half || (rem == half && (q & 1u))) q += 1;
  // value = q * 2^qexp; renormalise
  int ee = qexp;
  if (e >= -6) {
    if (q == 16) { q = 8; ee += 1; }  // carried into the next binade
    const int efield = (ee + 3) + 7;   // exponent of the leading bit + bias
    if (efield > 15 || (efield == 15 && (q - 8) > 6)) return static_cast<f8_t>(sign | 0x7eu);  // 448
    return static_cast<f8_t>(sign | (static_cast<uint32_t>(efield) << 3) | static_cast<uint32_t>(q - 8));
  }
  // subnormal region: q in 0..8 quanta of 2^-9 (8 = min normal 2^-6)
  if (q >= 8) return static_cast<f8_t>(sign | (1u << 3) | static_cast<uint32_t>(q - 8));
  return static_cast<f8_t>(sign | static_cast<uint32_t>(q));
}

__device__ __forceinline__ float f64_to_f32(double x) { return static_cast<float>(x); }

// ---------------------------------------------------------------- misc
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

inline size_t dtype_size(rt_dtype t) {
  switch (t) {
    case RT_F64: return 8;
    case RT_F32: return 4;
    case RT_BF16: return 2;
    case RT_F8E4M3: return 1;
  }
  return 0;
}

// Workgroup barrier ordering LDS only: it waits for this wave's LDS operations but
// not for its outstanding global loads, so prefetches stay in flight across it
// (__syncthreads also drains every global access of the wave).  Use only where
// the waves exchange data through LDS alone.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// 1/sqrt(x) for normal x > 0: hardware estimate refined by two Newton steps
// (each roughly doubles the correct bits), accurate to a few units in the last place.
__device__ __forceinline__ double rsq_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(x * y, y, -1.0);  // x y^2 - 1
    y = fma(-0.5 * y, e, y);
  }
  return y;
}


}  // namespace rt
