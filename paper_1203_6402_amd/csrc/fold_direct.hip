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

// Rows longer than 128 are processed in two halves so a point never needs
// more than 128 registers; the sum order over coordinates is the same.
// One thread per point (or per listed point).  The early exits keep the
// candidate-row addresses wave-uniform, so they are read with scalar loads.
template <int DP, typename T>
__global__ __launch_bounds__(kFoldBlock) void k_fold_direct(FoldArgs a) {
  constexpr int DCH = DP <= 128 ? DP : DP / 2;
  constexpr int NCH = DP / DCH;
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
  float nx = 0.0f;  // ||x||^2 when requested; stored after the candidate loop
  if constexpr (NCH == 1) {
    float x[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) x[j] = (j < d) ? Elem<T>::get(X, row + j, sc) : 0.0f;
    if (a.norms) {
#pragma unroll
      for (int j = 0; j < DP; ++j) nx = fmaf(x[j], x[j], nx);
    }
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
    if (a.norms) {
      for (int j = 0; j < d; ++j) {
        const float v = Elem<T>::get(X, row + j, sc);
        nx = fmaf(v, v, nx);
      }
    }
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
  // All global stores come after the candidate loop: a store before it could
  // alias the candidate rows and force them onto vector loads.
  if (a.norms) a.norms[i] = nx;
  if (a.first) {
    a.D2[i] = best;
    a.A[i] = bj >= 0 ? id0 + bj : -1;
  } else if (bj >= 0 && best < a.D2[i]) {
    a.D2[i] = best;
    a.A[i] = id0 + bj;
  }
}

// Direct-form rescan of the points a screen pass listed: one wave per point,
// each lane takes every 64th candidate; the wave reduction keeps the smallest
// distance and, among equal ones, the lowest id -- the decision the
// one-thread-per-point fold takes, with the same per-candidate arithmetic.
template <int DP, typename T>
__global__ __launch_bounds__(256) void k_rescan(FoldArgs a) {
  __shared__ float xs[4][DP];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int nlist = *a.list_len;
  int id0, m;
  if (a.rs) {
    id0 = a.rs[0];
    m = a.rs[1] - id0;
  } else {
    id0 = a.id0_host;
    m = a.m_host;
  }
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const float* __restrict__ C = a.C + (int64_t)id0 * DP;
  for (int it = blockIdx.x * 4 + w; it < nlist; it += gridDim.x * 4) {
    const int p = a.list[it];
    const float sc = row_scale_of<T>(a.row_scale, p);
    for (int e = lane; e < DP; e += 64) xs[w][e] = (e < a.d) ? Elem<T>::get(X, (int64_t)p * a.d + e, sc) : 0.0f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float best = INFINITY;
    int bj = -1;
    for (int c = lane; c < m; c += 64) {
      const float4* cr = reinterpret_cast<const float4*>(C + (int64_t)c * DP);
      float acc = 0.0f;
#pragma unroll
      for (int e4 = 0; e4 < DP / 4; ++e4) {
        const float4 cv = cr[e4];
        float t = xs[w][4 * e4 + 0] - cv.x;
        acc = fmaf(t, t, acc);
        t = xs[w][4 * e4 + 1] - cv.y;
        acc = fmaf(t, t, acc);
        t = xs[w][4 * e4 + 2] - cv.z;
        acc = fmaf(t, t, acc);
        t = xs[w][4 * e4 + 3] - cv.w;
        acc = fmaf(t, t, acc);
      }
      if (acc < best) {
        best = acc;
        bj = c;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float ob = __shfl_xor(best, off, 64);
      const int oj = __shfl_xor(bj, off, 64);
      if (ob < best || (ob == best && (unsigned)oj < (unsigned)bj)) {
        best = ob;
        bj = oj;
      }
    }
    if (lane == 0) {
      if (a.first) {
        a.D2[p] = best;
        a.A[p] = bj >= 0 ? id0 + bj : -1;
      } else if (bj >= 0 && best < a.D2[p]) {
        a.D2[p] = best;
        a.A[p] = id0 + bj;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ||x||^2 in FP32, coordinates in order (same arithmetic as the fold's norm).
template <typename T>
__global__ __launch_bounds__(256) void k_rownorm(const T* X, const float* row_scale, int n, int d,
                                                 float* norms) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float sc = row_scale_of<T>(row_scale, i);
  float nx = 0.0f;
  for (int j = 0; j < d; ++j) {
    const float v = Elem<T>::get(X, (int64_t)i * d + j, sc);
    nx = fmaf(v, v, nx);
  }
  norms[i] = nx;
}

hipError_t launch_rownorm(kmpar_dtype dt, const void* X, const float* row_scale, int n, int d,
                          float* norms, hipStream_t s) {
  const dim3 grid((n + 255) / 256), block(256);
  switch (dt) {
    case KMPAR_F32:
      hipLaunchKernelGGL(k_rownorm<float>, grid, block, 0, s, (const float*)X, row_scale, n, d, norms);
      break;
    case KMPAR_BF16:
      hipLaunchKernelGGL(k_rownorm<bf16_t>, grid, block, 0, s, (const bf16_t*)X, row_scale, n, d,
                         norms);
      break;
    case KMPAR_FP8_E4M3:
      hipLaunchKernelGGL(k_rownorm<fp8_t>, grid, block, 0, s, (const fp8_t*)X, row_scale, n, d, norms);
      break;
  }
  return hipGetLastError();
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

template <typename T>
static hipError_t launch_rescan_t(int DP, const FoldArgs& a, hipStream_t s) {
  int blocks = (a.list_cap + 3) / 4;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) return hipSuccess;
  const dim3 grid(blocks), block(256);
  switch (DP) {
#define KMPAR_CASE(V) \
  case V:             \
    hipLaunchKernelGGL((k_rescan<V, T>), grid, block, 0, s, a); break;
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

hipError_t launch_rescan(kmpar_dtype dt, int DP, const FoldArgs& a, hipStream_t s) {
  switch (dt) {
    case KMPAR_F32: return launch_rescan_t<float>(DP, a, s);
    case KMPAR_BF16: return launch_rescan_t<bf16_t>(DP, a, s);
    case KMPAR_FP8_E4M3: return launch_rescan_t<fp8_t>(DP, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace kmpar
