// Device helpers shared by the kmpar kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kmpar {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128-bit multiplies; round keys bumped by two Weyl constants.
// Only word 0 of the output block is used by the method.
// ---------------------------------------------------------------------------
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ULL;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ULL;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73BULL;

enum : uint64_t { kTagFirst = 1, kTagRound = 2, kTagRecluster = 3, kTagExact = 4 };

__device__ __forceinline__ uint64_t philox_word0(uint64_t seed, uint64_t tag, uint64_t a,
                                                 uint64_t b, uint64_t inst) {
  uint64_t c0 = a, c1 = b, c2 = inst, c3 = 0, k0 = seed, k1 = tag;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// U[0,1) with 53 random bits.
__device__ __forceinline__ double philox_uniform(uint64_t seed, uint64_t tag, uint64_t a,
                                                 uint64_t b, uint64_t inst) {
  return (double)(philox_word0(seed, tag, a, b, inst) >> 11) * 0x1.0p-53;
}

// Uniform integer in [0, n): high word of word0 * n.
__device__ __forceinline__ uint64_t philox_index(uint64_t seed, uint64_t tag, uint64_t a,
                                                 uint64_t b, uint64_t inst, uint64_t n) {
  return __umul64hi(philox_word0(seed, tag, a, b, inst), n);
}

// ---------------------------------------------------------------------------
// Element decoding.  All three storage types decode exactly into FP32 (BF16
// is the top half of an FP32; an e4m3 code has 4 significant bits and the
// row scale is applied with one rounding).
// ---------------------------------------------------------------------------
struct bf16_t {
  uint16_t bits;
};
struct fp8_t {
  uint8_t bits;
};

__device__ __forceinline__ float decode_bf16(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

// OCP FP8 e4m3 ("e4m3fn"): 1 sign, 4 exponent bits (bias 7), 3 mantissa bits,
// subnormals at exponent 0, the all-ones code is NaN, no infinities.
__device__ __forceinline__ float decode_e4m3(uint8_t q) {
  const uint32_t s = (uint32_t)(q & 0x80) << 24;
  const uint32_t e = (q >> 3) & 0xF;
  const uint32_t m = q & 0x7;
  float v;
  if (e == 0) {
    v = (float)m * 0x1.0p-9f;  // subnormal: m * 2^-6 / 8
  } else if (e == 0xF && m == 0x7) {
    v = __uint_as_float(0x7FC00000u);
  } else {
    v = __uint_as_float(((e + 120u) << 23) | (m << 20));  // 2^(e-7) * (1 + m/8)
  }
  return __uint_as_float(__float_as_uint(v) | s);
}

template <typename T>
struct Elem;
// get: element idx of X; from_bits: the same value from the element's raw
// bits (the low 8 * sizeof(T) bits of b), for kernels that load vectors.
template <>
struct Elem<float> {
  static __device__ __forceinline__ float get(const float* X, int64_t idx, float) { return X[idx]; }
  static __device__ __forceinline__ float from_bits(uint32_t b, float) { return __uint_as_float(b); }
};
template <>
struct Elem<bf16_t> {
  static __device__ __forceinline__ float get(const bf16_t* X, int64_t idx, float) {
    return decode_bf16(X[idx].bits);
  }
  static __device__ __forceinline__ float from_bits(uint32_t b, float) {
    return decode_bf16((uint16_t)b);
  }
};
// An FP8 element is fl(q * s): the product is rounded once, never fused into
// the arithmetic that uses it (every kernel then sees the same values).
template <>
struct Elem<fp8_t> {
  static __device__ __forceinline__ float from_bits(uint32_t b, float scale) {
#pragma clang fp contract(off)
    return decode_e4m3((uint8_t)b) * scale;
  }
  static __device__ __forceinline__ float get(const fp8_t* X, int64_t idx, float scale) {
    return from_bits(X[idx].bits, scale);
  }
};

template <typename T>
__device__ __forceinline__ float row_scale_of(const float* rs, int64_t i) {
  return 1.0f;
}
template <>
__device__ __forceinline__ float row_scale_of<fp8_t>(const float* rs, int64_t i) {
  return rs[i];
}

// ---------------------------------------------------------------------------
// Fixed-order reductions and scans (deterministic).
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  return v;  // valid in lane 0
}

// Block sum in a fixed tree order; the result is returned to every thread.
template <typename V, int BS>
__device__ __forceinline__ V block_sum(V v, V* sh) {
  constexpr int NW = BS / kWave;
  v = wave_sum(v);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  V t = V(0);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NW; ++i) t += sh[i];
    sh[NW] = t;
  }
  __syncthreads();
  return sh[NW];
}

// Inclusive scan within a wave (Hillis-Steele, fixed order).
template <typename V>
__device__ __forceinline__ V wave_incl_scan(V v) {
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    V o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

// One DPP step on an FP64 value (both 32-bit halves): lanes whose source is
// outside the row or whose row is masked off get 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Inclusive FP64 scan of a wave through DPP in a fixed order: prefix within
// each 16-lane row (shifts 1, 2, 4, 8), then row 15 and row 31 broadcasts
// carry the row totals forward.  Every lane of the wave must be active.
__device__ __forceinline__ double wave_incl_scan_f64(double v) {
  v += dpp_f64<0x111, 0xF>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xF>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xF>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xF>(v);  // row_shr:8
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}
// The value of lane l - 1 (0 in lane 0), by a whole-wave DPP shift.
__device__ __forceinline__ double wave_shr1_f64(double v) { return dpp_f64<0x138, 0xF>(v); }
// The value held by lane `src` (wave-uniform), via scalar reads.
__device__ __forceinline__ double wave_read_f64(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Exclusive block scan of one value per thread; *total receives the block sum.
// sh must hold BS/64 + 1 values.
template <typename V, int BS>
__device__ __forceinline__ V block_excl_scan(V v, V* sh, V* total) {
  constexpr int NW = BS / kWave;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  V inc = wave_incl_scan(v);
  V exc = __shfl_up(inc, 1, kWave);
  if (lane == 0) exc = V(0);
  __syncthreads();
  if (lane == kWave - 1) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    V run = V(0);
    for (int i = 0; i < NW; ++i) {
      V t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[NW] = run;
  }
  __syncthreads();
  V res = sh[w] + exc;
  *total = sh[NW];
  __syncthreads();
  return res;
}

}  // namespace kmpar
