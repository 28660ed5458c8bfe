// Distance fold in FP32 direct form (Algorithm 2 steps 4-5 as they act on
// d^2(x, C); Section 3.1 for assignment and cost).
//
// One thread owns one point and keeps its coordinates in registers; the m
// candidate rows are the same for every lane, so they are read with
// wave-uniform (scalar) loads and each lane does d subtract/FMA pairs per
// candidate.  Candidates are met in id order and a candidate replaces the
// current best only when strictly closer, so ties keep the lowest id.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace kmpar {

int padded_dim(int d) {
  if (d <= 64) return (d + 3) / 4 * 4;
  if (d <= 128) return (d + 15) / 16 * 16;
  return (d + 31) / 32 * 32;
}

template <int DP, typename T>
__global__ __launch_bounds__(kFoldBlock) void k_fold_direct(FoldArgs a) {
  // Rows longer than 128 are processed in two halves so the point never
  // needs more than 128 registers; the sum order over coordinates is the same.
  constexpr int DCH = DP <= 128 ? DP : DP / 2;
  constexpr int NCH = DP / DCH;
  static_assert(DP % DCH == 0, "padded dim must split into equal chunks");

  const int slot = blockIdx.x * kFoldBlock + threadIdx.x;
  int i;
  if (a.list) {
    if (slot >= *a.list_len) return;
    i = a.list[slot];
  } else {
    if (slot >= a.n) return;
    i = slot;
  }
  int id0, m;
  if (a.rs) {
    id0 = a.rs[0];
    m = a.rs[1] - id0;
  } else {
    id0 = a.id0_host;
    m = a.m_host;
  }
  const float* __restrict__ C = a.C + (int64_t)id0 * DP;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const float sc = row_scale_of<T>(a.row_scale, i);
  const int d = a.d;
  const int64_t row = (int64_t)i * d;

  float best = INFINITY;
  int bj = -1;
  if constexpr (NCH == 1) {
    float x[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) x[j] = (j < d) ? Elem<T>::get(X, row + j, sc) : 0.0f;
    for (int c = 0; c < m; ++c) {
      const float* __restrict__ cr = C + (int64_t)c * DP;
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < DP; ++j) {
        const float t = x[j] - cr[j];
        acc = fmaf(t, t, acc);
      }
      if (acc < best) {
        best = acc;
        bj = c;
      }
    }
  } else {
    constexpr int CB = 8;
    for (int c0 = 0; c0 < m; c0 += CB) {
      float acc[CB];
#pragma unroll
      for (int q = 0; q < CB; ++q) acc[q] = 0.0f;
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        float x[DCH];
#pragma unroll
        for (int j = 0; j < DCH; ++j) {
          const int jj = h * DCH + j;
          x[j] = (jj < d) ? Elem<T>::get(X, row + jj, sc) : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < CB; ++q) {
          if (c0 + q < m) {
            const float* __restrict__ cr = C + (int64_t)(c0 + q) * DP + h * DCH;
#pragma unroll
            for (int j = 0; j < DCH; ++j) {
              const float t = x[j] - cr[j];
              acc[q] = fmaf(t, t, acc[q]);
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < CB; ++q) {
        if (c0 + q < m && acc[q] < best) {
          best = acc[q];
          bj = c0 + q;
        }
      }
    }
  }
  if (a.first) {
    a.D2[i] = best;
    a.A[i] = bj >= 0 ? id0 + bj : -1;
  } else if (bj >= 0 && best < a.D2[i]) {
    a.D2[i] = best;
    a.A[i] = id0 + bj;
  }
}

template <typename T>
static hipError_t launch_t(int DP, const FoldArgs& a, hipStream_t s) {
  const int work = a.list ? a.list_cap : a.n;
  if (work <= 0) return hipSuccess;
  const dim3 grid((work + kFoldBlock - 1) / kFoldBlock), block(kFoldBlock);
  switch (DP) {
#define KMPAR_CASE(V) \
  case V:             \
    hipLaunchKernelGGL((k_fold_direct<V, T>), grid, block, 0, s, a); break;
    KMPAR_CASE(4) KMPAR_CASE(8) KMPAR_CASE(12) KMPAR_CASE(16) KMPAR_CASE(20) KMPAR_CASE(24)
    KMPAR_CASE(28) KMPAR_CASE(32) KMPAR_CASE(36) KMPAR_CASE(40) KMPAR_CASE(44) KMPAR_CASE(48)
    KMPAR_CASE(52) KMPAR_CASE(56) KMPAR_CASE(60) KMPAR_CASE(64) KMPAR_CASE(80) KMPAR_CASE(96)
    KMPAR_CASE(112) KMPAR_CASE(128) KMPAR_CASE(160) KMPAR_CASE(192) KMPAR_CASE(224)
    KMPAR_CASE(256)
#undef KMPAR_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fold_direct(kmpar_dtype dt, int DP, const FoldArgs& a, hipStream_t s) {
  switch (dt) {
    case KMPAR_F32: return launch_t<float>(DP, a, s);
    case KMPAR_BF16: return launch_t<bf16_t>(DP, a, s);
    case KMPAR_FP8_E4M3: return launch_t<fp8_t>(DP, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace kmpar
