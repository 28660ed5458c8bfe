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
#include "rows.hpp"

namespace kmpar {

// The fold of one pass into point i's state: (D2, A) move to the pass's
// best only when strictly closer (ties keep the lower id), and S, when kept,
// is the second-smallest distance over every candidate met so far.
// TRACK: the pass keeps S (a.S != nullptr); without it S is left alone.
template <bool TRACK = true>
__device__ __forceinline__ void fold_apply(const FoldArgs& a, int i, int id0, float best, int bj,
                                           float second) {
  if (a.first) {
    a.D2[i] = best;
    a.A[i] = bj >= 0 ? id0 + bj : -1;
    if constexpr (TRACK) a.S[i] = second;
  } else if (bj >= 0 && best < a.D2[i]) {
    if constexpr (TRACK) a.S[i] = fminf(a.D2[i], second);
    a.D2[i] = best;
    a.A[i] = id0 + bj;
  } else if (TRACK && bj >= 0) {
    a.S[i] = fminf(a.S[i], best);
  }
}

// A candidate at distance acc met in id order: the strictly smaller becomes
// the best (ties keep the earlier), the other bounds the second smallest
// (TRACK: only passes that keep S track it; the others spare its registers).
template <bool TRACK = true>
__device__ __forceinline__ void keep_two(float acc, int c, float& best, int& bj, float& second) {
  if (acc < best) {
    if constexpr (TRACK) second = best;
    best = acc;
    bj = c;
  } else if constexpr (TRACK) {
    second = fminf(second, acc);
  }
}

// Rows longer than 128 are processed in two halves so a point never needs
// more than 128 registers; the sum order over coordinates is the same.
// One thread per point (or per listed point).  The early exits keep the
// candidate-row addresses wave-uniform, so they are read with scalar loads.
template <int DP, typename T, bool TRACK>
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
  // candidates [c_lo, c_hi) of this block row's shard (all m unsharded)
  int c_lo = 0, c_hi = m;
  if (a.packed) {
    c_lo = (int)((int64_t)blockIdx.y * m / a.shards);
    c_hi = (int)((int64_t)(blockIdx.y + 1) * m / a.shards);
  }
  const float* __restrict__ C = a.C + (int64_t)id0 * DP;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const float sc = row_scale_of<T>(a.row_scale, i);
  const int d = a.d;
  const int64_t row = (int64_t)i * d;

  float best = INFINITY, second = INFINITY;
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
    for (int c = c_lo; c < c_hi; ++c) {
      const float* __restrict__ cr = C + (int64_t)c * DP;
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < DP; ++j) {
        const float t = x[j] - cr[j];
        acc = fmaf(t, t, acc);
      }
      keep_two<TRACK>(acc, c, best, bj, second);
    }
  } else {
    if (a.norms) {
      for (int j = 0; j < d; ++j) {
        const float v = Elem<T>::get(X, row + j, sc);
        nx = fmaf(v, v, nx);
      }
    }
    constexpr int CB = 8;
    for (int c0 = c_lo; c0 < c_hi; c0 += CB) {
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
          if (c0 + q < c_hi) {
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
      for (int q = 0; q < CB; ++q)
        if (c0 + q < c_hi) keep_two<TRACK>(acc[q], c0 + q, best, bj, second);
    }
  }
  // All global stores come after the candidate loop: a store before it could
  // alias the candidate rows and force them onto vector loads.
  if (a.norms) a.norms[i] = nx;
  if (a.packed) {
    // The reducer's minimum over the shards: distances are non-negative, so
    // their FP32 bits order as integers, and equal distances keep the lower id.
    if (bj >= 0)
      atomicMin(&a.packed[i], ((unsigned long long)__float_as_uint(best) << 32) |
                                  (unsigned long long)(unsigned)(id0 + bj));
    return;
  }
  fold_apply<TRACK>(a, i, id0, best, bj, second);
}

// Direct-form rescan of the points a screen pass listed.  A block takes 32
// listed points at a time (their decoded rows in LDS with an odd row stride)
// and streams the m candidates through LDS in chunks of 32 rows (row stride
// DP + 4, so the two rows a wave reads at once sit in different banks), each
// candidate row read once per 32 points.  Thread t serves point t % 32 and
// candidates s, s + 8, ... of every chunk, s = t / 32.  Each distance has
// the fold's arithmetic (t = x_e - c_e, acc = fma(t, t, acc), e ascending
// over the zero-padded row), each thread keeps its first strictly smallest
// candidate, and the eight slots' winners are merged by (distance, id): per
// point the smallest distance, the lowest id on ties, which is the decision
// the one-thread-per-point fold takes.
// A short list leaves most CUs idle, so when the groups of 32 points number
// at most half the grid, each group's candidates are cut into S slices of
// whole chunks (S a power of two, at most 8, with groups * S within the
// grid), one block per (group, slice); the slices' winners go to a.rpart and
// k_rescan_merge combines them in slice order by (distance, id), the same
// decision. Both kernels derive S from the device-side list length alone.

__device__ __forceinline__ int rescan_split(int groups, int grid, bool can_split) {
  int S = 1;
  if (can_split)
    while (S < kRescanMaxSplit && groups * S * 2 <= grid) S *= 2;
  return S;
}

// Keeps (b, j, s) as the better of itself and (ob, oj, os): smaller
// distance, then lower id (j = -1, no candidate, compares above every id);
// s, the second smallest, is the smallest of the rest.
__device__ __forceinline__ void rescan_better(float ob, int oj, float os, float& b, int& j,
                                              float& s) {
  if (ob < b || (ob == b && (unsigned)oj < (unsigned)j)) {
    s = fminf(fminf(s, b), os);
    b = ob;
    j = oj;
  } else {
    s = fminf(s, fminf(ob, os));
  }
}

template <int DP, typename T, bool TRACK>
__global__ __launch_bounds__(256) void k_rescan(FoldArgs a) {
  constexpr int P = kRescanPts, CC = kRescanCands, XS = DP + 1, CSTR = DP + 4;
  constexpr int NS = 256 / P, NI = CC / NS;  // candidate slots, candidates per slot
  constexpr int NV = (CC * (DP / 4) + 255) / 256;  // float4 of a chunk per thread
  // This thread's share of candidate rows c0 .. c0+CC-1 (zeros past m).
  auto load_chunk = [](const float* C, int c0, int m, float4 (&v)[NV]) {
    const int nc = min(CC, m - c0);
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int idx = threadIdx.x + u * 256;
      const int j = idx / (DP / 4), e4 = idx - j * (DP / 4);
      v[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (idx < CC * (DP / 4) && j < nc)
        v[u] = reinterpret_cast<const float4*>(C + (int64_t)(c0 + j) * DP)[e4];
    }
  };
  __shared__ float xs[P * XS];
  __shared__ __attribute__((aligned(16))) float cs[CC * CSTR];
  __shared__ float rb[NS][P];
  __shared__ int rj[NS][P];
  __shared__ float rs2[NS][P];
  const int r = threadIdx.x % P, slot = threadIdx.x / P;
  const int nlist = *a.list_len;
  const int groups = (nlist + P - 1) / P;
  const int S = rescan_split(groups, gridDim.x, a.rpart != nullptr);
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
  const int nch = (m + CC - 1) / CC;
  for (int it = blockIdx.x; it < groups * S; it += gridDim.x) {
    const int g = it / S, sl = it - g * S;
    const int np = min(P, nlist - g * P);
    // this slice's candidates: chunks [sl nch / S, (sl + 1) nch / S)
    const int cbeg = (sl * nch / S) * CC, cend = min(m, ((sl + 1) * nch / S) * CC);
    __syncthreads();  // the previous group is merged and written
    for (int idx = threadIdx.x; idx < P * DP; idx += 256) {
      const int q = idx / DP, e = idx - q * DP;
      float v = 0.0f;
      if (q < np && e < a.d) {
        const int p = a.list[g * P + q];
        v = Elem<T>::get(X, (int64_t)p * a.d + e, row_scale_of<T>(a.row_scale, p));
      }
      xs[q * XS + e] = v;
    }
    float best = INFINITY, second = INFINITY;
    int bj = -1;
    const float* xr = xs + r * XS;
    // Candidate chunks go global -> registers -> LDS; the next chunk's loads
    // are issued before the current chunk is computed.
    float4 pre[NV];
    if (cbeg < cend) load_chunk(C, cbeg, cend, pre);
    for (int c0 = cbeg; c0 < cend; c0 += CC) {
      const int nc = min(CC, cend - c0);
      __syncthreads();  // the previous chunk is consumed (and xs is written)
#pragma unroll
      for (int u = 0; u < NV; ++u) {
        const int idx = threadIdx.x + u * 256;
        if (idx < CC * (DP / 4)) {
          const int j = idx / (DP / 4), e4 = idx - j * (DP / 4);
          reinterpret_cast<float4*>(cs + j * CSTR)[e4] = pre[u];
        }
      }
      __syncthreads();
      if (c0 + CC < cend) load_chunk(C, c0 + CC, cend, pre);
      float acc[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i) acc[i] = 0.0f;
#pragma unroll 2
      for (int e = 0; e < DP; e += 4) {
        const float x0 = xr[e], x1 = xr[e + 1], x2 = xr[e + 2], x3 = xr[e + 3];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          const float4 cv = reinterpret_cast<const float4*>(cs + (slot + NS * i) * CSTR)[e / 4];
          float t = x0 - cv.x;
          acc[i] = fmaf(t, t, acc[i]);
          t = x1 - cv.y;
          acc[i] = fmaf(t, t, acc[i]);
          t = x2 - cv.z;
          acc[i] = fmaf(t, t, acc[i]);
          t = x3 - cv.w;
          acc[i] = fmaf(t, t, acc[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int j = slot + NS * i;
        if (j < nc) keep_two<TRACK>(acc[i], c0 + j, best, bj, second);
      }
    }
    rb[slot][r] = best;
    rj[slot][r] = bj;
    if constexpr (TRACK) rs2[slot][r] = second;
    __syncthreads();
    if (slot == 0 && r < np) {
      for (int q = 1; q < NS; ++q)
        rescan_better(rb[q][r], rj[q][r], TRACK ? rs2[q][r] : INFINITY, best, bj, second);
      if (S == 1)
        fold_apply<TRACK>(a, a.list[g * P + r], id0, best, bj, second);
      else
        a.rpart[(int64_t)it * P + r] =
            make_int4(__float_as_int(best), bj, TRACK ? __float_as_int(second) : 0x7F800000, 0);
    }
  }
}

// Merges the slices of a split rescan (nothing to do when S = 1). grid is the
// rescan's launch grid, from which S is derived again.
template <bool TRACK>
__global__ __launch_bounds__(256) void k_rescan_merge(FoldArgs a, int grid) {
  constexpr int P = kRescanPts;
  const int nlist = *a.list_len;
  const int groups = (nlist + P - 1) / P;
  const int S = rescan_split(groups, grid, a.rpart != nullptr);
  if (S == 1) return;
  const int id0 = a.rs ? a.rs[0] : a.id0_host;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nlist; i += gridDim.x * 256) {
    const int g = i / P, r = i - g * P;
    float best = INFINITY, second = INFINITY;
    int bj = -1;
    for (int sl = 0; sl < S; ++sl) {
      const int4 v = a.rpart[(int64_t)(g * S + sl) * P + r];
      rescan_better(__int_as_float(v.x), v.y, __int_as_float(v.z), best, bj, second);
    }
    fold_apply<TRACK>(a, a.list[i], id0, best, bj, second);
  }
}

// Assignment passes against few centers (rows of up to 64 padded elements)
// read X once and do little arithmetic per byte: they are bound by HBM, where
// k_fold_direct's one thread per point issues d strided loads per lane and
// keeps few bytes in flight.  Two forms, each folding every candidate with
// the FMA chain of k_fold_direct (candidates in id order, ties to the lower
// id), so the result is k_fold_direct's bit for bit.  No list, no norms, no
// runner-up.
//
// m <= kStreamMaxM: one wave of 64 points per block, whose rows (one
// contiguous span) are copied into LDS by direct 16-byte global-to-LDS loads
// that hold no registers while in flight; many small blocks per CU keep the
// most bytes in flight.  Each lane then reads its row from LDS and folds the
// candidates.  The one partial wave at the end of X copies its rows lane by
// lane.
typedef __attribute__((address_space(3))) void fold_lds_void;
typedef const __attribute__((address_space(1))) void fold_gbl_void;

template <int DP, typename T>
__global__ __launch_bounds__(64) void k_fold_stream(FoldArgs a) {
  constexpr int S = (int)sizeof(T);
  __shared__ __attribute__((aligned(16))) char rows[64 * DP * S];  // the wave's 64 raw rows
  const int lane = threadIdx.x, d = a.d, rowb = d * S;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int64_t p = p0 + lane;
  const bool full = p0 + 64 <= a.n;  // the whole span lies inside X
  const bool live = p < a.n;
  if (full) {
    const int bytes = 64 * rowb;  // a multiple of 16
    const char* src = static_cast<const char*>(a.X) + p0 * rowb;
    for (int v0 = 0; v0 < bytes; v0 += 1024)
      if (v0 + 16 * lane < bytes)
        __builtin_amdgcn_global_load_lds((fold_gbl_void*)(src + v0 + 16 * lane),
                                         (fold_lds_void*)(rows + v0), 16, 0, 0);
  } else if (live) {  // the partial wave: each lane copies its own row
    const T* X = static_cast<const T*>(a.X);
    for (int j = 0; j < d; ++j) reinterpret_cast<T*>(rows)[lane * d + j] = X[p * d + j];
  }
  const float sc = live ? row_scale_of<T>(a.row_scale, p) : 1.0f;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (!live) return;
  float x[DP];
  const T* xr = reinterpret_cast<const T*>(rows + lane * rowb);
#pragma unroll
  for (int j = 0; j < DP; ++j) x[j] = j < d ? Elem<T>::get(xr, j, sc) : 0.0f;
  const int m = a.m_host, id0 = a.id0_host;
  const float* __restrict__ C = a.C + (int64_t)id0 * DP;
  float best = INFINITY, second = INFINITY;
  int bj = -1;
  for (int c = 0; c < m; ++c) {
    const float* __restrict__ cr = C + (int64_t)c * DP;
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < DP; ++j) {
      const float t = x[j] - cr[j];
      acc = fmaf(t, t, acc);
    }
    keep_two<false>(acc, c, best, bj, second);
  }
  fold_apply<false>(a, (int)p, id0, best, bj, second);
}

// kStreamMaxM < m <= kStagedMaxM: blocks of four waves stage their 64 rows
// through LDS with coalesced 16-byte loads (the first pass's staging), and
// the waves split the candidates (wave w takes c = w, w + 4, ...), each
// keeping the nearest of its share; the four are merged in candidate order
// (smaller distance, then lower id).
template <int DP, typename T>
__global__ __launch_bounds__(256) void k_fold_few(FoldArgs a) {
  __shared__ float xs[64 * (DP + 1)];  // [64][XS], XS = d + 1 when d is a multiple of 32
  __shared__ float ss[64];             // FP8 row scales
  __shared__ float rb[4][64];
  __shared__ int rj[4][64];
  const int d = a.d, pad = d % 32 == 0 ? 1 : 0, XS = d + pad;
  const int p0 = blockIdx.x * 64;
  const int np = max(0, min(64, a.n - p0));
  stage_rows<T>(static_cast<const T*>(a.X), a.row_scale, p0, np, d, pad, ss, xs);
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), pl = threadIdx.x % 64;
  float x[DP];
#pragma unroll
  for (int j = 0; j < DP; ++j) x[j] = (j < d && pl < np) ? xs[pl * XS + j] : 0.0f;
  const int m = a.m_host, id0 = a.id0_host;
  const float* __restrict__ C = a.C + (int64_t)id0 * DP;
  float best = INFINITY, second = INFINITY;
  int bj = -1;
  for (int c = w; c < m; c += 4) {
    const float* __restrict__ cr = C + (int64_t)c * DP;
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < DP; ++j) {
      const float t = x[j] - cr[j];
      acc = fmaf(t, t, acc);
    }
    keep_two<false>(acc, c, best, bj, second);
  }
  rb[w][pl] = best;
  rj[w][pl] = bj;
  __syncthreads();
  if (w != 0 || pl >= np) return;
#pragma unroll
  for (int q = 1; q < 4; ++q) {
    const float ob = rb[q][pl];
    const int oj = rj[q][pl];
    if (ob < best || (ob == best && (unsigned)oj < (unsigned)bj)) {
      best = ob;
      bj = oj;
    }
  }
  fold_apply<false>(a, p0 + pl, id0, best, bj, second);
}

// The fold for rows of more than 128 padded elements (no list, no norms),
// each row split over W = ceil(DP / 64) waves: a block of 128 W threads holds its
// kSplitPts = 128 points in two groups of W waves, wave s of a group keeping elements
// [64 s, min(64 s + 64, DP)) of its 64 points' rows in registers, decoded
// once. Per chunk of CH candidates, stage s continues the FMA chain of stage
// s - 1 (a partial sum left in LDS, double buffered, one chunk behind) over
// its elements and the last stage keeps the best candidate; one barrier per
// step of the pipeline. The chain and the candidate order are the fold's, so
// the result is bitwise the same. Read in halves by one thread, such rows
// were re-read and re-decoded every 8 candidates (n = 50M rows of 256 FP8
// elements, k = 2000: a PLAIN init took 121 s, 10.6 s split). Rows of 65 to
// 128 elements use the two-wave form below (k_fold_pair), whose registers
// allow seven waves per SIMD (n = 16M rows of 128 BF16 elements, k = 1000: a
// PLAIN init 1.6 s with whole rows in one thread, 0.7 s).
constexpr int kSplitPts = 128;                 // points per block of k_fold_split
constexpr int kSplitGroups = kSplitPts / 64;   // waves per pipeline stage

template <int DP, typename T, bool TRACK>
__device__ __forceinline__ void fold_split_body(const FoldArgs& a) {
  constexpr int W = (DP + 63) / 64;
  constexpr int CH = 8;
  static_assert(W >= 3 && W <= 4, "rows of 129 to 256 padded elements");
  __shared__ float part[2][CH][W - 1][kSplitPts];  // [buffer][candidate][stage][point]
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  // pipeline stage: elements [64 st, 64 st + 64); the same for the whole
  // wave, which readfirstlane tells the compiler, so that the candidate rows
  // are read with scalar loads rather than 64 lanes' vector loads
  const int st = __builtin_amdgcn_readfirstlane(wv / kSplitGroups);
  const int pl = (wv % kSplitGroups) * kWave + lane;  // the point within the block
  const int i = blockIdx.x * kSplitPts + pl;
  const bool live = i < a.n;                  // every wave takes part in the barriers
  int id0, m;
  if (a.rs) {
    id0 = a.rs[0];
    m = a.rs[1] - id0;
  } else {
    id0 = a.id0_host;
    m = a.m_host;
  }
  const float* __restrict__ C = a.C + (int64_t)id0 * DP + st * 64;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const float sc = live ? row_scale_of<T>(a.row_scale, i) : 1.0f;
  const int d = a.d;
  const int64_t row = (int64_t)i * d;
  const int e0 = st * 64;
  constexpr int NL = DP - 64 * (W - 1);       // elements of the last stage
  float x[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) x[j] = (live && e0 + j < d) ? Elem<T>::get(X, row + e0 + j, sc) : 0.0f;
  float best = INFINITY;
  int bj = -1;
  float second = INFINITY;
  const int nch = (m + CH - 1) / CH;
  for (int it = 0; it < nch + W - 1; ++it) {
    const int c = it - st;                    // the chunk this stage takes now
    if (c >= 0 && c < nch) {
      const int c0 = c * CH, nc = min(CH, m - c0);
      const int b = c & 1;
      if (st == W - 1) {
        for (int jj = 0; jj < nc; ++jj) {
          const float* __restrict__ cr = C + (int64_t)(c0 + jj) * DP;
          float acc = part[b][jj][W - 2][pl];
#pragma unroll
          for (int e = 0; e < NL; ++e) {
            const float t = x[e] - cr[e];
            acc = fmaf(t, t, acc);
          }
          keep_two<TRACK>(acc, c0 + jj, best, bj, second);
        }
      } else {
        for (int jj = 0; jj < nc; ++jj) {
          const float* __restrict__ cr = C + (int64_t)(c0 + jj) * DP;
          float acc = st == 0 ? 0.0f : part[b][jj][st - 1][pl];
#pragma unroll
          for (int e = 0; e < 64; ++e) {
            const float t = x[e] - cr[e];
            acc = fmaf(t, t, acc);
          }
          part[b][jj][st][pl] = acc;
        }
      }
    }
    __syncthreads();  // stage outputs of this step visible; inputs of the last step consumed
  }
  if (st != W - 1 || !live) return;
  fold_apply<TRACK>(a, i, id0, best, bj, second);
}

template <int DP, typename T>
__global__ __launch_bounds__(kSplitPts * ((DP + 63) / 64)) void k_fold_split(FoldArgs a) {
  fold_split_body<DP, T, false>(a);
}
// Tracking the runner-up costs a register; held to six waves per SIMD (three
// blocks of eight waves per CU) as the plain variant runs.
template <int DP, typename T>
__global__ __launch_bounds__(kSplitPts * ((DP + 63) / 64)) __attribute__((amdgpu_waves_per_eu(6)))
void k_fold_split_track(FoldArgs a) {
  fold_split_body<DP, T, true>(a);
}

// The fold for rows of 65 to 128 padded elements (no list, no norms), each
// row split over two waves: a block of 2 * kFoldBlock threads holds its 256
// points in four pairs of waves, the first wave of a pair with elements
// [0, 64) of its 64 rows in registers, the second with [64, DP). Per chunk
// of 16 candidates the first wave runs the FMA chain over its elements and
// leaves each partial sum in LDS; one chunk later the second wave continues
// the chain over the rest of the row and keeps the best candidate. Same chain
// and candidate order as k_fold_direct, so the result is bitwise the same.
template <int DP, typename T, bool TRACK>
__device__ __forceinline__ void fold_pair_body(const FoldArgs& a) {
  static_assert(DP > 64 && DP <= 128, "rows of 65 to 128 padded elements");
  constexpr int H1 = DP - 64, CH = 16;
  __shared__ float part[2][CH][kFoldBlock];  // [buffer][candidate of the chunk][point]
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int half = wv / 4;                    // 0: elements [0, 64); 1: [64, DP)
  const int pl = (wv % 4) * kWave + lane;     // the point within the block
  const int i = blockIdx.x * kFoldBlock + pl;
  const bool live = i < a.n;                  // every wave takes part in the barriers
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
  const float sc = live ? row_scale_of<T>(a.row_scale, i) : 1.0f;
  const int d = a.d;
  const int64_t row = (int64_t)i * d;
  const int e0 = half ? 64 : 0;
  float x[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) x[j] = (live && e0 + j < d) ? Elem<T>::get(X, row + e0 + j, sc) : 0.0f;
  float best = INFINITY, second = INFINITY;
  int bj = -1;
  const int nch = (m + CH - 1) / CH;
  for (int it = 0; it <= nch; ++it) {
    if (half == 0) {
      if (it < nch) {
        const int c0 = it * CH, nc = min(CH, m - c0);
        float* dst = &part[it & 1][0][pl];
        for (int jj = 0; jj < nc; ++jj) {
          const float* __restrict__ cr = C + (int64_t)(c0 + jj) * DP;
          float acc = 0.0f;
#pragma unroll
          for (int e = 0; e < 64; ++e) {
            const float t = x[e] - cr[e];
            acc = fmaf(t, t, acc);
          }
          dst[jj * kFoldBlock] = acc;
        }
      }
    } else if (it > 0) {
      const int c0 = (it - 1) * CH, nc = min(CH, m - c0);
      const float* src = &part[(it - 1) & 1][0][pl];
      for (int jj = 0; jj < nc; ++jj) {
        const float* __restrict__ cr = C + (int64_t)(c0 + jj) * DP + 64;
        float acc = src[jj * kFoldBlock];
#pragma unroll
        for (int e = 0; e < H1; ++e) {
          const float t = x[e] - cr[e];
          acc = fmaf(t, t, acc);
        }
        keep_two<TRACK>(acc, c0 + jj, best, bj, second);
      }
    }
    __syncthreads();  // chunk it written, chunk it - 1 consumed
  }
  if (half == 0 || !live) return;
  fold_apply<TRACK>(a, i, id0, best, bj, second);
}

template <int DP, typename T>
__global__ __launch_bounds__(2 * kFoldBlock) void k_fold_pair(FoldArgs a) {
  fold_pair_body<DP, T, false>(a);
}
// Tracking the runner-up: held to seven waves per SIMD as the plain variant.
template <int DP, typename T>
__global__ __launch_bounds__(2 * kFoldBlock) __attribute__((amdgpu_waves_per_eu(7)))
void k_fold_pair_track(FoldArgs a) {
  fold_pair_body<DP, T, true>(a);
}

template <typename T, bool TRACK>
static hipError_t launch_t(int DP, const FoldArgs& a, hipStream_t s) {
  const int work = a.list ? a.list_cap : a.n;
  if (work <= 0) return hipSuccess;
  if (a.packed && (a.list || a.norms || a.shards < 1)) return hipErrorInvalidValue;
  const dim3 grid((work + kFoldBlock - 1) / kFoldBlock, a.packed ? a.shards : 1), block(kFoldBlock);
  if (a.packed) {  // every row length through the one-thread-per-point fold
    switch (DP) {
#define KMPAR_SHARD(V) \
  case V: hipLaunchKernelGGL((k_fold_direct<V, T, TRACK>), grid, block, 0, s, a); return hipGetLastError();
      KMPAR_SHARD(4) KMPAR_SHARD(8) KMPAR_SHARD(12) KMPAR_SHARD(16) KMPAR_SHARD(20)
      KMPAR_SHARD(24) KMPAR_SHARD(28) KMPAR_SHARD(32) KMPAR_SHARD(36) KMPAR_SHARD(40)
      KMPAR_SHARD(44) KMPAR_SHARD(48) KMPAR_SHARD(52) KMPAR_SHARD(56) KMPAR_SHARD(60)
      KMPAR_SHARD(64) KMPAR_SHARD(80) KMPAR_SHARD(96) KMPAR_SHARD(112) KMPAR_SHARD(128)
      KMPAR_SHARD(160) KMPAR_SHARD(192) KMPAR_SHARD(224) KMPAR_SHARD(256)
#undef KMPAR_SHARD
      default: return hipErrorInvalidValue;
    }
  }
  if (!a.list && !a.norms && DP > 64 && DP <= 128) {
    switch (DP) {
#define KMPAR_PAIR(V)                                                             \
  case V:                                                                  \
    if constexpr (TRACK)                                                        \
      hipLaunchKernelGGL((k_fold_pair_track<V, T>), grid, dim3(2 * kFoldBlock), 0, s, a); \
    else                                                                        \
      hipLaunchKernelGGL((k_fold_pair<V, T>), grid, dim3(2 * kFoldBlock), 0, s, a); \
    return hipGetLastError();
      KMPAR_PAIR(80) KMPAR_PAIR(96) KMPAR_PAIR(112) KMPAR_PAIR(128)
#undef KMPAR_PAIR
      default: break;
    }
  }
  if (!a.list && !a.norms && !a.packed && !a.S && !a.rs && a.m_host <= kStagedMaxM && DP <= 64) {
    switch (DP) {
#define KMPAR_STAGED(V)                                                                     \
  case V:                                                                                   \
    if (a.m_host <= kStreamMaxM)                                                            \
      hipLaunchKernelGGL((k_fold_stream<V, T>), dim3((a.n + 63) / 64), dim3(64), 0, s, a); \
    else                                                                                    \
      hipLaunchKernelGGL((k_fold_few<V, T>), dim3((a.n + 63) / 64), dim3(256), 0, s, a);   \
    return hipGetLastError();
      KMPAR_STAGED(4) KMPAR_STAGED(8) KMPAR_STAGED(12) KMPAR_STAGED(16) KMPAR_STAGED(20)
      KMPAR_STAGED(24) KMPAR_STAGED(28) KMPAR_STAGED(32) KMPAR_STAGED(36) KMPAR_STAGED(40)
      KMPAR_STAGED(44) KMPAR_STAGED(48) KMPAR_STAGED(52) KMPAR_STAGED(56) KMPAR_STAGED(60)
      KMPAR_STAGED(64)
#undef KMPAR_STAGED
      default: break;
    }
  }
  if (!a.list && !a.norms && DP > 128) {
    switch (DP) {
#define KMPAR_SPLIT(V)                                                            \
  case V:                                                                  \
    if constexpr (TRACK)                                                        \
      hipLaunchKernelGGL((k_fold_split_track<V, T>), dim3((work + kSplitPts - 1) / kSplitPts), \
                         dim3(kSplitPts * ((V + 63) / 64)), 0, s, a);                     \
    else                                                                        \
      hipLaunchKernelGGL((k_fold_split<V, T>), dim3((work + kSplitPts - 1) / kSplitPts), \
                         dim3(kSplitPts * ((V + 63) / 64)), 0, s, a);                     \
    return hipGetLastError();
      KMPAR_SPLIT(160) KMPAR_SPLIT(192) KMPAR_SPLIT(224) KMPAR_SPLIT(256)
#undef KMPAR_SPLIT
      default: break;
    }
  }
  switch (DP) {
#define KMPAR_CASE(V) \
  case V:             \
    hipLaunchKernelGGL((k_fold_direct<V, T, TRACK>), grid, block, 0, s, a); break;
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

__global__ __launch_bounds__(256) void k_unpack_min(const unsigned long long* packed, int n, int* A,
                                                    float* D2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const unsigned long long v = packed[i];
  A[i] = (int)(unsigned)(v & 0xFFFFFFFFull);
  if (D2) D2[i] = __uint_as_float((unsigned)(v >> 32));
}

hipError_t launch_unpack_min(const unsigned long long* packed, int n, int* A, float* D2,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_min, dim3((n + 255) / 256), dim3(256), 0, s, packed, n, A, D2);
  return hipGetLastError();
}

// Passes that keep each point's runner-up distance (a.S) run the tracking
// variants; the others (assignment passes) the lighter ones.
hipError_t launch_fold_direct(kmpar_dtype dt, int DP, const FoldArgs& a, hipStream_t s) {
  const bool track = a.S != nullptr;
  switch (dt) {
    case KMPAR_F32: return track ? launch_t<float, true>(DP, a, s) : launch_t<float, false>(DP, a, s);
    case KMPAR_BF16: return track ? launch_t<bf16_t, true>(DP, a, s) : launch_t<bf16_t, false>(DP, a, s);
    case KMPAR_FP8_E4M3: return track ? launch_t<fp8_t, true>(DP, a, s) : launch_t<fp8_t, false>(DP, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, bool TRACK>
static hipError_t launch_rescan_t(int DP, const FoldArgs& a, hipStream_t s) {
  // the listed count is only known on the device: enough blocks for the
  // largest list up to four per CU, each looping over groups of points
  int blocks = (a.list_cap + kRescanPts - 1) / kRescanPts;
  if (blocks > kRescanMaxItems) blocks = kRescanMaxItems;
  if (blocks < 1) return hipSuccess;
  const dim3 grid(blocks), block(256);
  switch (DP) {
#define KMPAR_CASE(V) \
  case V:             \
    hipLaunchKernelGGL((k_rescan<V, T, TRACK>), grid, block, 0, s, a); break;
    KMPAR_CASE(4) KMPAR_CASE(8) KMPAR_CASE(12) KMPAR_CASE(16) KMPAR_CASE(20) KMPAR_CASE(24)
    KMPAR_CASE(28) KMPAR_CASE(32) KMPAR_CASE(36) KMPAR_CASE(40) KMPAR_CASE(44) KMPAR_CASE(48)
    KMPAR_CASE(52) KMPAR_CASE(56) KMPAR_CASE(60) KMPAR_CASE(64) KMPAR_CASE(80) KMPAR_CASE(96)
    KMPAR_CASE(112) KMPAR_CASE(128) KMPAR_CASE(160) KMPAR_CASE(192) KMPAR_CASE(224)
    KMPAR_CASE(256)
#undef KMPAR_CASE
    default:
      return hipErrorInvalidValue;
  }
  if (a.rpart) {
    const int mb = (min(a.list_cap, kRescanMaxItems * kRescanPts) + 255) / 256;
    hipLaunchKernelGGL(k_rescan_merge<TRACK>, dim3(mb), dim3(256), 0, s, a, blocks);
  }
  return hipGetLastError();
}

hipError_t launch_rescan(kmpar_dtype dt, int DP, const FoldArgs& a, hipStream_t s) {
  switch (dt) {
    case KMPAR_F32:
      return a.S ? launch_rescan_t<float, true>(DP, a, s) : launch_rescan_t<float, false>(DP, a, s);
    case KMPAR_BF16:
      return a.S ? launch_rescan_t<bf16_t, true>(DP, a, s) : launch_rescan_t<bf16_t, false>(DP, a, s);
    case KMPAR_FP8_E4M3:
      return a.S ? launch_rescan_t<fp8_t, true>(DP, a, s) : launch_rescan_t<fp8_t, false>(DP, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace kmpar
