// Coalesced staging of blocks of rows of X into LDS (shared by the screen's
// first pass and operand preparation and by the k-means++ steps).
#pragma once

#include "common.hpp"

namespace kmpar {

// Rows whose screen operands are codes with a separate per-row scale.
template <typename T>
struct ScaledRows {
  static constexpr bool value = false;
};
template <>
struct ScaledRows<fp8_t> {
  static constexpr bool value = true;
};

// ------------------------------------------------------------ row staging
// Rows p0 .. p0+np-1 of X decoded to FP32 into xs[row * XS + col], XS = d + pad.
// The block's rows are one contiguous span starting 16-byte aligned (64 d
// sizeof(T) bytes per block): coalesced 16-byte loads, four in flight per
// thread, each decoded into 16 / sizeof(T) elements; a tail shorter than 16
// bytes is read element by element. FP8 rows' scales go to ss first. Every
// thread of the block calls it; the caller synchronises before reading xs.
template <typename T>
__device__ __forceinline__ void stage_rows(const T* X, const float* row_scale, int p0, int np, int d,
                                           int pad, float* ss, float* xs) {
  constexpr bool SC = ScaledRows<T>::value;
  if constexpr (SC) {
    if (threadIdx.x < np) ss[threadIdx.x] = row_scale[p0 + threadIdx.x];
    __syncthreads();
  }
  constexpr int S = (int)sizeof(T), EPV = 16 / S;
  const int cnt = np * d;
  const int nvec = cnt * S / 16;
  const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(X) +
                                                    (int64_t)p0 * d * S);
  constexpr int U = 4;
  for (int v0 = 0; v0 < nvec; v0 += U * 256) {
    uint4 w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = v0 + u * 256 + threadIdx.x;
      if (idx < nvec) w[u] = src[idx];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = v0 + u * 256 + threadIdx.x;
      if (idx < nvec) {
        const uint32_t wd[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
        const int e = idx * EPV;
        int row = e / d, col = e - row * d;
#pragma unroll
        for (int k = 0; k < EPV; ++k) {
          const uint32_t b = wd[(k * S) / 4] >> (8 * ((k * S) % 4));
          xs[e + k + row * pad] = Elem<T>::from_bits(b, SC ? ss[row] : 1.0f);
          if (++col == d) {
            col = 0;
            ++row;
          }
        }
      }
    }
  }
  for (int e = nvec * EPV + threadIdx.x; e < cnt; e += 256)
    xs[e + (e / d) * pad] = Elem<T>::get(X, (int64_t)p0 * d + e, row_scale_of<T>(row_scale, p0 + e / d));
}

}  // namespace kmpar
