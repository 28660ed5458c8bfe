// The passes of k-means|| around the distance fold: first center, cost phi,
// Bernoulli draws with order-preserving compaction, candidate gather, the
// Step-7 weight histogram, the Step-8 weighted k-means++ recluster and the
// Lloyd centroid update.  Every reduction and scan runs in a fixed order, so
// results are bit-reproducible.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "recluster_block.hpp"

namespace kmpar {

#define KMPAR_RET_LAST() return hipGetLastError()

// --------------------------------------------------------------- first center
// Algorithm 2 step 1: the first center is point Index(n) of the FIRST stream.
__global__ void k_first(int n, uint64_t seed, uint64_t inst, int* cand_point, int* rs,
                        kmpar_stats* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int i0 = (int)philox_index(seed, kTagFirst, 0, 0, inst, (uint64_t)n);
  cand_point[0] = i0;
  rs[0] = 0;
  rs[1] = 1;
  st->round_count[0] = 1;
  st->status = KMPAR_OK;
  st->n_rescanned = 0;
  st->flagged_draws = 0;
  st->flagged_picks = 0;
  st->flagged_argmins = 0;
}

hipError_t launch_first(int n, uint64_t seed, uint64_t inst, int* cand_point, int* rs,
                        kmpar_stats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_first, dim3(1), dim3(64), 0, s, n, seed, inst, cand_point, rs, st);
  KMPAR_RET_LAST();
}

// --------------------------------------------------------------------- gather
// Copies the m_t rows kept in round t into the row-major candidate buffer
// Call[id][DP] (read by the folds and the recluster), zero-padded past d.
template <typename T>
__global__ void k_gather(const T* X, const float* row_scale, int d, int DP, const int* cand_point,
                         const int* rs, int t, float* Call, float* CallT, int ldT) {
  const int id0 = rs[t];
  const int m = rs[t + 1] - id0;
  const int j = blockIdx.x;
  if (j >= m) return;
  const int c = id0 + j;
  const int p = cand_point[c];
  const float sc = row_scale_of<T>(row_scale, p);
  for (int e = threadIdx.x; e < DP; e += blockDim.x) {
    const float v = (e < d) ? Elem<T>::get(X, (int64_t)p * d + e, sc) : 0.0f;
    Call[(int64_t)c * DP + e] = v;
    if (CallT && e < d) CallT[(int64_t)e * ldT + c] = v;
  }
}

hipError_t launch_gather(kmpar_dtype dt, const void* X, const float* row_scale, int d, int DP,
                         const int* cand_point, const int* rs, int t, int cap_round, float* Call,
                         float* CallT, int ldT, hipStream_t s) {
  const dim3 grid(cap_round), block(64);
  switch (dt) {
    case KMPAR_F32:
      hipLaunchKernelGGL(k_gather<float>, grid, block, 0, s, (const float*)X, row_scale, d, DP,
                         cand_point, rs, t, Call, CallT, ldT);
      break;
    case KMPAR_BF16:
      hipLaunchKernelGGL(k_gather<bf16_t>, grid, block, 0, s, (const bf16_t*)X, row_scale, d, DP,
                         cand_point, rs, t, Call, CallT, ldT);
      break;
    case KMPAR_FP8_E4M3:
      hipLaunchKernelGGL(k_gather<fp8_t>, grid, block, 0, s, (const fp8_t*)X, row_scale, d, DP,
                         cand_point, rs, t, Call, CallT, ldT);
      break;
  }
  KMPAR_RET_LAST();
}

// Pads m rows of length d into rows of length DP.
__global__ void k_pad_rows(const float* C, int m, int d, int DP, float* Cpad) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * DP) return;
  const int r = (int)(idx / DP), e = (int)(idx % DP);
  Cpad[idx] = (e < d) ? C[(int64_t)r * d + e] : 0.0f;
}

hipError_t launch_pad_rows(const float* C, int m, int d, int DP, float* Cpad, hipStream_t s) {
  const int64_t tot = (int64_t)m * DP;
  hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, C, m, d,
                     DP, Cpad);
  KMPAR_RET_LAST();
}

// ------------------------------------------------------------------ cost phi
// phi = sum_i D2_i in FP64: fixed chunks per block, fixed tree per block, then
// one block sums the block partials in order (Section 3.5: per-partition
// partial costs summed by one reducer).
__global__ __launch_bounds__(256) void k_phi_partial(const float* D2, int n, double* part) {
  __shared__ double sh[8];
  const int base = blockIdx.x * kPhiChunk;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < kPhiChunk / 256; ++r) {
    const int i = base + r * 256 + threadIdx.x;
    if (i < n) acc += (double)D2[i];
  }
  const double tot = block_sum<double, 256>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_phi_final(const double* part, int nb, double* out) {
  __shared__ double sh[8];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  const double tot = block_sum<double, 256>(acc, sh);
  if (threadIdx.x == 0) *out = tot;
}

hipError_t launch_phi(const float* D2, int n, double* part, double* out, hipStream_t s) {
  const int nb = (n + kPhiChunk - 1) / kPhiChunk;
  hipLaunchKernelGGL(k_phi_partial, dim3(nb), dim3(256), 0, s, D2, n, part);
  hipLaunchKernelGGL(k_phi_final, dim3(1), dim3(256), 0, s, part, nb, out);
  KMPAR_RET_LAST();
}

// ---------------------------------------------------------------------- draw
__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x % kWave;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint64_t lanemask_gt() {
  const int lane = threadIdx.x % kWave;
  return lane == kWave - 1 ? 0ull : (~0ull << (lane + 1));
}

// Algorithm 2 step 4: point i is kept in round t iff u < p with
// p = min(1, ell * D2_i / phi) and u = U(seed, ROUND, (i, t, inst)).
// *flag is set when |u - p| <= band * p: a draw that D^2 within its FP32
// error band could have decided the other way.
__device__ __forceinline__ int keep_point(const float* D2, int i, double phi, double ell,
                                          uint64_t seed, int t, uint64_t inst, double band,
                                          int* flag) {
  *flag = 0;
  if (!(phi > 0.0)) return 0;
  double p = ell * (double)D2[i] / phi;
  if (p > 1.0) p = 1.0;
  const double u = philox_uniform(seed, kTagRound, (uint64_t)i, (uint64_t)t, inst);
  *flag = (p > 0.0 && fabs(u - p) <= band * p) ? 1 : 0;
  return u < p ? 1 : 0;
}

// Masks of kept points per block: word j covers points base + 64 j + lane.
constexpr int kDrawMasks = kDrawChunk / 64;

// Counts the points a block keeps and records them as one ballot per wave and
// 64 points, so the write pass needs neither D^2 nor the draws again.
__global__ __launch_bounds__(256) void k_draw_count(const float* D2, int n, const double* phi,
                                                    double ell, uint64_t seed, int t,
                                                    uint64_t inst, double band, int* cnt,
                                                    uint64_t* keep, kmpar_stats* st) {
  __shared__ int sh[8];
  const double ph = *phi;
  const int base = blockIdx.x * kDrawChunk;
  const int w = threadIdx.x / kWave;
  int c = 0, nf = 0;
#pragma unroll
  for (int r = 0; r < kDrawChunk / 256; ++r) {
    const int i = base + r * 256 + threadIdx.x;
    int fl = 0;
    const int kp = (i < n) ? keep_point(D2, i, ph, ell, seed, t, inst, band, &fl) : 0;
    c += kp;
    nf += fl;
    const uint64_t b = __ballot(kp);
    if (threadIdx.x % kWave == 0) keep[(int64_t)blockIdx.x * kDrawMasks + r * 4 + w] = b;
  }
  const int tot = block_sum<int, 256>(c, sh);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
  const int ftot = block_sum<int, 256>(nf, sh);
  if (threadIdx.x == 0 && ftot) atomicAdd(&st->flagged_draws, ftot);
}

// In-place exclusive scan of a[0..L) by one block; *total = sum.  With rs,
// it also commits round t: m_t = min(total, cap), rs[t+1] = rs[t] + m_t.
__global__ __launch_bounds__(1024) void k_scan1(int* a, int L, int* total, int* rs, int t, int cap,
                                                kmpar_stats* st) {
  __shared__ long long sh[17];
  const int R = (L + 1023) / 1024;
  const int lo = min(L, (int)threadIdx.x * R), hi = min(L, lo + R);
  long long s = 0;
  for (int j = lo; j < hi; ++j) s += a[j];
  long long tot;
  long long run = block_excl_scan<long long, 1024>(s, sh, &tot);
  for (int j = lo; j < hi; ++j) {
    const int v = a[j];
    a[j] = (int)run;
    run += v;
  }
  if (threadIdx.x == 0 && total) *total = (int)tot;
  if (threadIdx.x == 0 && rs) {
    const int m = tot < cap ? (int)tot : cap;
    rs[t + 1] = rs[t] + m;
    st->round_count[t] = m;
    if (tot > cap) st->status = KMPAR_E_OVERFLOW;
  }
}

// Writes the kept point indices in increasing point order, ranked from the
// block's masks.
__global__ __launch_bounds__(256) void k_draw_write(const uint64_t* keep, const int* off,
                                                    const int* rs, int t, int cap,
                                                    int* cand_point) {
  __shared__ uint64_t m[kDrawMasks];
  __shared__ int pre[kDrawMasks];
  if (threadIdx.x < kDrawMasks) m[threadIdx.x] = keep[(int64_t)blockIdx.x * kDrawMasks + threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int j = 0; j < kDrawMasks; ++j) {
      pre[j] = run;
      run += __popcll(m[j]);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int run0 = off[blockIdx.x], start = rs[t];
  for (int r = 0; r < kDrawMasks / 4; ++r) {
    const int j = r * 4 + w;
    const uint64_t mk = m[j];
    if ((mk >> lane) & 1) {
      const int pos = run0 + pre[j] + __popcll(mk & lanemask_lt());
      if (pos < cap) cand_point[start + pos] = blockIdx.x * kDrawChunk + j * kWave + lane;
    }
  }
}

hipError_t launch_draw(const float* D2, int n, const double* phi, double ell, uint64_t seed, int t,
                       uint64_t inst, double band, int* cnt, uint64_t* keep, int* scan_total,
                       int* rs, int cap_round, int* cand_point, kmpar_stats* st, hipStream_t s) {
  const int nb = (n + kDrawChunk - 1) / kDrawChunk;
  hipLaunchKernelGGL(k_draw_count, dim3(nb), dim3(256), 0, s, D2, n, phi, ell, seed, t, inst, band,
                     cnt, keep, st);
  return launch_round_compact(n, cnt, keep, scan_total, rs, t, cap_round, cand_point, st, s);
}

hipError_t launch_round_compact(int n, int* cnt, const uint64_t* keep, int* scan_total, int* rs,
                                int t, int cap_round, int* cand_point, kmpar_stats* st,
                                hipStream_t s) {
  const int nb = (n + kDrawChunk - 1) / kDrawChunk;
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, s, cnt, nb, scan_total, rs, t, cap_round, st);
  hipLaunchKernelGGL(k_draw_write, dim3(nb), dim3(256), 0, s, keep, cnt, rs, t, cap_round,
                     cand_point);
  KMPAR_RET_LAST();
}

// Points whose nearest candidate has a runner-up within the FP32 band:
// S <= (1 + band) D2 (a tie at zero included).
__global__ __launch_bounds__(256) void k_flag_argmins(const float* D2, const float* S, int n,
                                                      double band, kmpar_stats* st) {
  __shared__ int sh[8];
  int c = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    c += ((double)S[i] <= (1.0 + band) * (double)D2[i]) ? 1 : 0;
  const int tot = block_sum<int, 256>(c, sh);
  if (threadIdx.x == 0 && tot) atomicAdd(&st->flagged_argmins, tot);
}

hipError_t launch_flag_argmins(const float* D2, const float* S, int n, double band,
                               kmpar_stats* st, hipStream_t s) {
  const int grid = std::min((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_flag_argmins, dim3(grid), dim3(256), 0, s, D2, S, n, band, st);
  KMPAR_RET_LAST();
}

__global__ void k_finish_rounds(const int* rs, int rounds, kmpar_stats* st) {
  if (threadIdx.x == 0) st->n_candidates = rs[rounds + 1];
}

hipError_t launch_finish_rounds(const int* rs, int rounds, kmpar_stats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_rounds, dim3(1), dim3(64), 0, s, rs, rounds, st);
  KMPAR_RET_LAST();
}

// ------------------------------------------------------------ fills / copies
__global__ void k_fill_i32(int* p, int v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}
hipError_t launch_fill_i32(int* p, int v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v,
                     count);
  KMPAR_RET_LAST();
}
__global__ void k_copy_i32(const int* src, int* dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}
hipError_t launch_copy_i32(const int* src, int* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, src, dst,
                     count);
  KMPAR_RET_LAST();
}

// ------------------------------------------------------------- Step 7 weights
// w_c = |{i : A_i = c}|, counted in LDS per block, then merged with integer
// atomics (exact, so the result does not depend on their order).  A is read
// four values per 16-byte load with four loads in flight per thread.
__global__ __launch_bounds__(256) void k_hist_lds(const int* A, int n, int* w, int nbins) {
  extern __shared__ int h[];
  for (int b = threadIdx.x; b < nbins; b += 256) h[b] = 0;
  __syncthreads();
  const int n4 = n / 4;
  const int4* A4 = reinterpret_cast<const int4*>(A);
  const int stride = gridDim.x * 256;
  constexpr int U = 4;
  for (int i0 = blockIdx.x * 256 + threadIdx.x; i0 < n4; i0 += U * stride) {
    int4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = i0 + u * stride;
      v[u] = idx < n4 ? A4[idx] : make_int4(-1, -1, -1, -1);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int a[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (a[q] >= 0 && a[q] < nbins) atomicAdd(&h[a[q]], 1);
    }
  }
  for (int i = 4 * n4 + blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const int a = A[i];
    if (a >= 0 && a < nbins) atomicAdd(&h[a], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += 256)
    if (h[b]) atomicAdd(&w[b], h[b]);
}

__global__ __launch_bounds__(256) void k_hist_global(const int* A, int n, int* w, int nbins) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const int a = A[i];
    if (a >= 0 && a < nbins) atomicAdd(&w[a], 1);
  }
}

// A block's LDS histogram may take up to this much of a CU's 160 KB (one
// block per CU above 80 KB, two below).
constexpr int kLdsBudget = 156 * 1024;

hipError_t launch_hist(const int* A, int n, int* w, int nbins, int num_cu, hipStream_t s) {
  hipError_t e = launch_fill_i32(w, 0, nbins, s);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)nbins * 4;
  if (lds <= (size_t)kLdsBudget) {
    const int blocks = std::max(1, num_cu) * (lds <= 80 * 1024 ? 2 : 1);
    e = hipFuncSetAttribute((const void*)k_hist_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hist_lds, dim3(blocks), dim3(256), lds, s, A, n, w, nbins);
  } else {
    hipLaunchKernelGGL(k_hist_global, dim3(512), dim3(256), 0, s, A, n, w, nbins);
  }
  KMPAR_RET_LAST();
}

// ---------------------------------------------------------- Step 8 recluster
// Weighted k-means++ (Algorithm 1 with weights) on the candidates, spread
// over G workgroups.  Block b holds candidates [b*m/G, (b+1)*m/G) -- rows,
// E and w -- in LDS.  Pick 0 has probability w_j / sum w (integer sums, exact
// in FP64); pick s >= 1 has probability w_j E_j / T with E_j the FP32
// direct-form distance to the nearest earlier pick and every sum in FP64.
// Pick s takes the smallest j whose running sum (block order, then thread
// runs, then candidate order) exceeds u*T, u = U(seed, RECL, (s, 0, inst)).
//
// Per pick s, two hops between workgroups and no barrier counter:
//  1. every block waits for the row of pick s-1 (polling the elements of its
//     row slot), folds it into E, and publishes its FP64 partial in its
//     partial slot of round s;
//  2. every block polls the G partials of round s and derives T and the
//     owner of u*T in block order; the owner finds the pick and publishes its
//     row.
// Every round has slots of its own, all-ones until written (partials are
// finite, rows of finite inputs never have that bit pattern), so a slot is
// written once and read by polling that word alone: agent-scope atomic
// coherence is all the exchange needs, with no fences (on this chip an
// agent-scope release or acquire writes back or invalidates the L2).  Every
// wait has a spin limit, so every wave exits (status KMPAR_E_HIP).
constexpr int kReclBlock = 512;
constexpr unsigned kSpinLimit = 1u << 22;
constexpr size_t kReclLdsBudget = 144 * 1024;
constexpr unsigned long long kEmpty64 = ~0ull;
constexpr unsigned kEmpty32 = ~0u;

__device__ __forceinline__ unsigned long long poll64(const double* p, int* failed) {
  const auto* q = reinterpret_cast<const unsigned long long*>(p);
  unsigned long long v;
  unsigned spins = 0;
  while ((v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == kEmpty64) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      *failed = 1;
      break;
    }
  }
  return v;
}
__device__ __forceinline__ unsigned poll32(const float* p, int* failed) {
  const auto* q = reinterpret_cast<const unsigned*>(p);
  unsigned v;
  unsigned spins = 0;
  while ((v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == kEmpty32) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      *failed = 1;
      break;
    }
  }
  return v;
}

struct ReclArgs {
  const float* Call;   // candidate rows, DP-padded
  int DP;
  int d;
  const int* w;
  const int* rs_end;   // device: number of candidates m
  int k;
  uint64_t seed;
  uint64_t inst;
  int fit;             // candidates per block at most (LDS capacity)
  const double* u;     // [k] the draws U(seed, RECL, (s, 0, inst))
  double* part;        // [k][G] partial slots, all-ones on entry
  float* prow;         // [k][DP] row slots of the picks, all-ones on entry
  int* picks;          // [k] output: candidate ids
  float* centers;      // [k][d] output rows
  kmpar_stats* st;
  double band;         // FP32 band of the distances (see pick_near_end)
  int xstride;         // workgroup b of the recluster is workgroup b * xstride of the grid
};

// The recluster's draws, one thread each, ahead of the sequential picks.
__global__ void k_recl_draws(uint64_t seed, uint64_t inst, int k, double* u) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < k) u[s] = philox_uniform(seed, kTagRecluster, (uint64_t)s, 0, inst);
}

// LROWS: the slice's rows sit in LDS (odd stride); otherwise they are read
// from Call in global memory (candidate sets too large for the CUs' LDS).
template <bool LROWS>
__global__ __launch_bounds__(kReclBlock) void k_recluster_grid(ReclArgs a) {
  extern __shared__ float4 lds4[];  // 16-byte aligned: cp is read as float4
  float* lds = reinterpret_cast<float*>(lds4);
  __shared__ double wtot[kReclBlock / kWave];
  __shared__ double gpart[kReclMaxBlocks];
  __shared__ double sh_u, sh_base, sh_top, sh_plo, sh_phi;
  __shared__ int sh_pick, sh_owner, sh_failed, sh_stop, sh_pflag;
  constexpr int NW = kReclBlock / kWave;
  // only every xstride-th workgroup takes part (see launch_recluster)
  if (blockIdx.x % a.xstride) return;
  const int b = blockIdx.x / a.xstride, tid = threadIdx.x, DP = a.DP, d = a.d;
  const int lane = tid % kWave, wv = tid / kWave;
  const int DL = LROWS ? DP + 1 : DP;  // odd LDS row stride: rows land in different banks
  const int m = *a.rs_end;
  // the blocks the candidate count needs (the grid is sized for the capacity)
  const int G = min((int)gridDim.x / a.xstride, (m + a.fit - 1) / a.fit);
  if (b >= G) return;
  const int lo = (int)((int64_t)b * m / G), hi = (int)((int64_t)(b + 1) * m / G);
  const int ns = hi - lo;
  float* cp = lds;                                               // [DP] row of the latest pick
  float* rows = LROWS ? cp + DP : nullptr;                       // [fit][DL]
  float* E = cp + DP + (LROWS ? (size_t)a.fit * DL : 0);         // [fit]
  int* wl = reinterpret_cast<int*>(E + a.fit);                   // [fit]
  const float* grows = a.Call + (int64_t)lo * DP;                // the slice in global memory
  if (tid == 0) {
    sh_failed = 0;
    sh_stop = 0;
  }
  if constexpr (LROWS) {
    for (int idx = tid; idx < ns * DP; idx += kReclBlock) {
      const int j = idx / DP, e = idx - j * DP;
      rows[j * DL + e] = grows[idx];
    }
  }
  for (int j = tid; j < ns; j += kReclBlock) wl[j] = a.w[lo + j];
  // each thread owns a contiguous run of the slice (one candidate when the
  // slice fits the block), so thread order is candidate order
  const int R = (ns + kReclBlock - 1) / kReclBlock;
  const int rlo = min(ns, tid * R), rhi = min(ns, rlo + R);
  int made = 0;
  for (int s = 0; s < a.k; ++s) {
    // the draw of this pick, loaded while the row of the previous one is in
    // flight
    const double u = a.u[s];
    if (s > 0) {
      // hop 2 of round s-1: the row of pick s-1
      if (tid < DP) cp[tid] = __uint_as_float(poll32(&a.prow[(int64_t)(s - 1) * DP + tid], &sh_failed));
      __syncthreads();
      if (sh_failed) break;
      // Direct form over the DP-padded row (the padding adds fmaf(0, 0, acc)
      // = acc), sixteen elements per step with the LDS reads issued first;
      // reads past the row stay inside the block's LDS and are masked.
      for (int j = rlo; j < rhi; ++j) {
        float acc = 0.0f;
        for (int e0 = 0; e0 < DP; e0 += 16) {
          float xr[16];
          float4 c4[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) c4[q] = reinterpret_cast<const float4*>(cp + e0)[q];
          if constexpr (LROWS) {
            const float* r = rows + (size_t)j * DL;
#pragma unroll
            for (int q = 0; q < 16; ++q) xr[q] = r[e0 + q];
          } else {
            // whole float4s of the DP-padded row only: no read past it
            const float4* r4 = reinterpret_cast<const float4*>(grows + (size_t)j * DP + e0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float4 v = (e0 + 4 * q < DP) ? r4[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
              xr[4 * q] = v.x;
              xr[4 * q + 1] = v.y;
              xr[4 * q + 2] = v.z;
              xr[4 * q + 3] = v.w;
            }
          }
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const float cq = q % 4 == 0 ? c4[q / 4].x : q % 4 == 1 ? c4[q / 4].y
                           : q % 4 == 2 ? c4[q / 4].z : c4[q / 4].w;
            const float t = e0 + q < DP ? xr[q] - cq : 0.0f;
            acc = fmaf(t, t, acc);
          }
        }
        E[j] = (s == 1) ? acc : fminf(E[j], acc);
      }
    }
    // this thread's mass (candidate order), its exclusive prefix in the
    // block and the block total, all in one fixed order
    double v = 0.0;
    for (int j = rlo; j < rhi; ++j) v += (s == 0) ? (double)wl[j] : (double)wl[j] * (double)E[j];
    const double inc = wave_incl_scan_f64(v);
    const double exw = wave_shr1_f64(inc);
    if (lane == kWave - 1) wtot[wv] = inc;
    __syncthreads();
    double wbase = 0.0, tot = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      if (q < wv) wbase += wtot[q];
      tot += wtot[q];
    }
    const double ex = wbase + exw;
    if (tid == 0)
      __hip_atomic_store(reinterpret_cast<unsigned long long*>(&a.part[(int64_t)s * G + b]),
                         (unsigned long long)__double_as_longlong(tot), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    // hop 1 of round s: all partials
    for (int q = tid; q < G; q += kReclBlock)
      gpart[q] = __longlong_as_double((long long)poll64(&a.part[(int64_t)s * G + q], &sh_failed));
    __syncthreads();
    if (wv == 0) {
      // T and the owner of u*T in block order: lane l sums a contiguous run
      // of partials, then a fixed-order wave scan (the same in every block)
      const int RG = (G + kWave - 1) / kWave;
      const int q0 = min(G, lane * RG), q1 = min(G, q0 + RG);
      double ls = 0.0;
      for (int q = q0; q < q1; ++q) ls += gpart[q];
      const double linc = wave_incl_scan_f64(ls);
      const double T = wave_read_f64(linc, kWave - 1);
      double run = wave_shr1_f64(linc);
      const double thr = u * T;
      int own = -1, last_pos = -1;
      double lo_b = 0.0, hi_b = 0.0;
      for (int q = q0; q < q1; ++q) {
        const double g = gpart[q];
        const double nxt = (q + 1 < G) ? run + g : T;
        if (g > 0.0) last_pos = q;
        if (own < 0 && run <= thr && thr < nxt && g > 0.0) {
          own = q;
          lo_b = run;
          hi_b = nxt;
        }
        run += g;
      }
      const uint64_t found = __ballot(own >= 0);
      int last = last_pos;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) last = max(last, __shfl_xor(last, off, kWave));
      if (found) {
        const int fl = __ffsll((unsigned long long)found) - 1;
        own = __shfl(own, fl, kWave);
        lo_b = __shfl(lo_b, fl, kWave);
        hi_b = __shfl(hi_b, fl, kWave);
      }
      if (lane == 0) {
        if (!(T > 0.0) || sh_failed) {
          sh_stop = 1;
        } else if (!found) {  // thr at or past the total by rounding
          own = last;
          lo_b = hi_b = INFINITY;
        }
        sh_owner = own;
        sh_base = lo_b;
        sh_top = hi_b;
        sh_u = thr;
        sh_pick = 0x7fffffff;
        sh_pflag = 0;
      }
    }
    __syncthreads();
    if (sh_stop) break;
    if (sh_owner == b) {
      const double thr = sh_u, base = sh_base;
      // The picked interval [lo, hi) of the running sums (recorded by the
      // thread that found the pick) decides whether u*T lay within the band
      // of one of its ends; a pick made by a rounding fallback always is.
      int my_pick = -1;
      double my_lo = 0.0, my_hi = 0.0;
      if (isinf(base)) {
        // rounding fallback: the last candidate with positive mass
        if (tid == 0) {
          for (int j = ns - 1; j >= 0; --j) {
            const double g = (s == 0) ? (double)wl[j] : (double)wl[j] * (double)E[j];
            if (g > 0.0) {
              sh_pick = j;
              break;
            }
          }
          sh_pflag = 1;
        }
      } else {
        const double b0 = base + ex;
        const double b1 = (tid + 1 < kReclBlock) ? b0 + v : sh_top;
        if (v > 0.0 && b0 <= thr && thr < b1) {
          double run = b0;
          int pick = -1, last = -1;
          for (int j = rlo; j < rhi; ++j) {
            const double g = (s == 0) ? (double)wl[j] : (double)wl[j] * (double)E[j];
            const double before = run;
            run += g;
            if (g > 0.0) last = j;
            if (g > 0.0 && run > thr) {
              pick = j;
              my_lo = before;
              my_hi = run;
              break;
            }
          }
          if (pick < 0) {  // u*T at the end of this run by rounding
            pick = last;
            my_lo = my_hi = thr;
          }
          my_pick = pick;
          if (pick >= 0) atomicMin(&sh_pick, pick);
        }
      }
      __syncthreads();
      if (my_pick >= 0 && my_pick == sh_pick) {
        sh_plo = my_lo;
        sh_phi = my_hi;
      }
      __syncthreads();
      if (sh_pick == 0x7fffffff) {
        // Thread-run bounds and the block bound come from different FP64
        // association orders; if no run claimed u*T, walk the slice in order.
        if (tid == 0) {
          double run = base;
          int last = -1;
          for (int j = 0; j < ns; ++j) {
            const double g = (s == 0) ? (double)wl[j] : (double)wl[j] * (double)E[j];
            const double before = run;
            run += g;
            if (g > 0.0) last = j;
            if (g > 0.0 && run > thr) {
              sh_pick = j;
              sh_plo = before;
              sh_phi = run;
              break;
            }
          }
          if (sh_pick == 0x7fffffff) {
            sh_pick = last;
            sh_pflag = 1;
          }
        }
        __syncthreads();
      }
      if (tid == 0 && (sh_pflag || pick_near_end(thr, sh_plo, sh_phi, a.band)))
        atomicAdd(&a.st->flagged_picks, 1);
      const int jl = sh_pick;
      // hop 2 of round s: publish the row, then the outputs
      const float* pr = LROWS ? rows + (size_t)jl * DL : grows + (size_t)jl * DP;
      if (tid < DP)
        __hip_atomic_store(reinterpret_cast<unsigned*>(&a.prow[(int64_t)s * DP + tid]),
                           __float_as_uint(pr[tid]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int e = tid; e < d; e += kReclBlock) a.centers[(int64_t)s * d + e] = pr[e];
      if (tid == 0) a.picks[s] = lo + jl;
    }
    made = s + 1;
  }
  if (b == 0 && tid == 0) {
    a.st->n_centers = made;
    if (sh_failed) a.st->status = KMPAR_E_HIP;
    else if (made < a.k && a.st->status == KMPAR_OK) a.st->status = KMPAR_E_TOOFEW;
  }
}

// Single-instance recluster in one 1024-thread workgroup (no grid barriers).
__global__ __launch_bounds__(1024) void k_recluster_block(const float* CallT, int ldT, int d,
                                                          const int* w, const int* rs_end, int k,
                                                          uint64_t seed, uint64_t inst, int* picks,
                                                          float* centers, kmpar_stats* st,
                                                          int cap_lds, double band) {
  extern __shared__ float lds[];
  recluster_block<1024>(CallT, ldT, d, w, *rs_end, k, seed, inst, picks, centers, st, lds, cap_lds,
                        band);
}

size_t recluster_block_lds(int capT, int k) { return (size_t)capT * 8 + (size_t)k * 8; }

hipError_t launch_recluster_block(const float* CallT, int capT, int d, const int* w,
                                  const int* rs_end, int k, uint64_t seed, uint64_t inst,
                                  int* picks, float* centers, kmpar_stats* st, double band,
                                  hipStream_t s) {
  const size_t lds = recluster_block_lds(capT, k);
  hipError_t e = hipFuncSetAttribute((const void*)k_recluster_block,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_recluster_block, dim3(1), dim3(1024), lds, s, CallT, capT, d, w, rs_end, k,
                     seed, inst, picks, centers, st, capT, band);
  KMPAR_RET_LAST();
}

bool recluster_plan(int capT, int DP, int num_cu, bool global_rows, ReclPlan* p) {
  // Slices of at most one candidate per thread with their rows in LDS (odd
  // stride); when the CUs cannot hold every slice that way, all CUs take
  // slices whose rows stay in global memory.  Every block must be resident
  // at once, so the grid never exceeds the CU count.
  const int gmax = std::min(num_cu, kReclMaxBlocks);
  const size_t head = (size_t)DP * 4;
  const size_t per_l = (size_t)(DP + 1) * 4 + 8;
  int fit = (int)std::min<size_t>(kReclBlock, (kReclLdsBudget - head) / per_l);
  int G = (capT + fit - 1) / fit;
  if (!global_rows && G <= gmax) {
    *p = ReclPlan{G, fit, true, head + (size_t)fit * per_l, num_cu};
    return true;
  }
  // global rows: one candidate per thread while the CUs suffice
  G = std::min(gmax, (capT + kReclBlock - 1) / kReclBlock);
  fit = (capT + G - 1) / G;
  const size_t lds = head + (size_t)fit * 8;
  if (lds > kReclLdsBudget) return false;
  *p = ReclPlan{G, fit, false, lds, num_cu};
  return true;
}

hipError_t launch_recluster(const float* Call, int DP, int d, const int* w, const int* rs_end,
                            int k, uint64_t seed, uint64_t inst, const ReclPlan& plan,
                            double* udraw, double* part, float* prow, int* picks,
                            float* centers, kmpar_stats* st, double band, hipStream_t s) {
  const int G = plan.G;
  hipLaunchKernelGGL(k_recl_draws, dim3((k + 255) / 256), dim3(256), 0, s, seed, inst, k, udraw);
  // every slot starts empty (all-ones); fill kernels, not memsets, so the
  // sequence can be captured in a graph
  hipError_t e = launch_fill_i32(reinterpret_cast<int*>(part), -1, 2 * (int64_t)k * G, s);
  if (e != hipSuccess) return e;
  e = launch_fill_i32(reinterpret_cast<int*>(prow), -1, (int64_t)k * DP, s);
  if (e != hipSuccess) return e;
  ReclArgs a;
  a.Call = Call;
  a.DP = DP;
  a.d = d;
  a.w = w;
  a.rs_end = rs_end;
  a.k = k;
  a.seed = seed;
  a.inst = inst;
  a.fit = plan.fit;
  a.u = udraw;
  a.part = part;
  a.prow = prow;
  a.picks = picks;
  a.centers = centers;
  a.st = st;
  a.band = band;
  // Workgroups are dealt to the XCDs in turn (workgroup i to XCD i mod 8),
  // so when the recluster needs at most one XCD's CUs, a grid of 8 G
  // workgroups of which every eighth takes part keeps its exchanges within
  // one XCD's L2; the others exit at once.
  a.xstride = G * kXcds <= plan.num_cu ? kXcds : 1;
  const void* fn = plan.lds_rows ? (const void*)k_recluster_grid<true>
                                 : (const void*)k_recluster_grid<false>;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan.lds);
  if (e != hipSuccess) return e;
  const int grid = G * a.xstride;
  if (plan.lds_rows)
    hipLaunchKernelGGL(k_recluster_grid<true>, dim3(grid), dim3(kReclBlock), plan.lds, s, a);
  else
    hipLaunchKernelGGL(k_recluster_grid<false>, dim3(grid), dim3(kReclBlock), plan.lds, s, a);
  KMPAR_RET_LAST();
}

// ------------------------------------------------------------- Lloyd update
// Deterministic centroid update (Section 3.1 centroid; Section 1 Lloyd):
//  1. per-block cluster counts   bcnt[c * nbs + b], c = 0 .. k, where key k
//     collects the points without a valid center (an assignment outside
//     [0, k), which only a point with no finite distance gets): they are
//     sorted behind every cluster and summed into none
//  2. exclusive scan of the flattened table -> each (cluster, block) slot
//  3. stable scatter of point indices into cluster-sorted order
//  4. cluster chunks of kSegChunk sorted points, each split into fixed
//     consecutive slices summed in FP64 in point order, the slices then
//     added in slice order
//  5. per cluster: its chunk sums added in fixed consecutive slices, each in
//     chunk order, the slices then in slice order; divided by the count.
// Every sum runs in an order fixed by (n, d, k, assignment) alone, so the
// update is reproducible run to run.
// The sort key of an assignment: the cluster, or k for none.
__device__ __forceinline__ int sort_key(int a, int k) { return (a >= 0 && a < k) ? a : k; }

__global__ __launch_bounds__(256) void k_sort_count(const int* A, int n, int k, int* bcnt,
                                                    int nbs) {
  extern __shared__ int h[];  // k + 1 keys
  for (int c = threadIdx.x; c <= k; c += 256) h[c] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortChunk;
  for (int r = threadIdx.x; r < kSortChunk; r += 256) {
    const int i = base + r;
    if (i < n) atomicAdd(&h[sort_key(A[i], k)], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c <= k; c += 256) bcnt[(int64_t)c * nbs + blockIdx.x] = h[c];
}

// Three-phase exclusive scan of a[0..L): tile sums, scan of the tile sums,
// tile-local scans plus offsets.
__global__ __launch_bounds__(256) void k_scan_tiles(const int* a, int64_t L, int* tsum) {
  __shared__ int sh[8];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int s = 0;
  for (int r = threadIdx.x; r < kScanTile; r += 256) {
    const int64_t j = base + r;
    if (j < L) s += a[j];
  }
  const int tot = block_sum<int, 256>(s, sh);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_apply(int* a, int64_t L, const int* toff) {
  __shared__ int sh[8];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int run = toff[blockIdx.x];
  for (int r = 0; r < kScanTile; r += 256) {
    const int64_t j = base + r + threadIdx.x;
    const int v = (j < L) ? a[j] : 0;
    int tot;
    const int ex = block_excl_scan<int, 256>(v, sh, &tot);
    if (j < L) a[j] = run + ex;
    run += tot;
  }
}

// One wave per block scatters its chunk in point order, a 64-point tile at a
// time; the keys of kSortAhead tiles are loaded before the first of them is
// placed. The lanes holding the same key are found with one ballot per key bit
// (nbits = bits of k, keys 0 .. k); a lane's slot is its key's cursor plus the
// number of lower lanes with that key, and the highest such lane advances the
// cursor by the group's size once every lane has read it.  Every point of
// the chunk gets a slot, so sorted[0 .. n) is written whole.
static_assert(kSortChunk % (64 * kSortAhead) == 0, "sort chunk must hold whole key batches");

__global__ __launch_bounds__(64) void k_sort_scatter(const int* A, int n, int k, int nbits,
                                                     const int* bbase, int nbs, int* sorted) {
  extern __shared__ int cur[];  // k + 1 keys
  for (int c = threadIdx.x; c <= k; c += 64) cur[c] = bbase[(int64_t)c * nbs + blockIdx.x];
  __syncthreads();
  const int base = blockIdx.x * kSortChunk;
  for (int t0 = 0; t0 < kSortChunk && base + t0 < n; t0 += 64 * kSortAhead) {
    int keys[kSortAhead];
#pragma unroll
    for (int u = 0; u < kSortAhead; ++u) {
      const int i = base + t0 + u * 64 + threadIdx.x;
      keys[u] = (i < n) ? sort_key(A[i], k) : -1;
    }
#pragma unroll
    for (int u = 0; u < kSortAhead; ++u) {
      const int i0 = base + t0 + u * 64;
      if (i0 >= n) break;
      const int i = i0 + threadIdx.x;
      const int key0 = keys[u];
      const bool valid = key0 >= 0;  // i < n
      const int key = valid ? key0 : 0;
      uint64_t grp = __ballot(valid);
      for (int b = 0; b < nbits; ++b) {
        const bool bit = (key >> b) & 1;
        const uint64_t on = __ballot(valid && bit);
        grp &= bit ? on : ~on;
      }
      const int pos0 = valid ? cur[key] : 0;
      __syncthreads();
      if (valid) {
        sorted[pos0 + __popcll(grp & lanemask_lt())] = i;
        if ((grp & lanemask_gt()) == 0) cur[key] = pos0 + __popcll(grp);
      }
      __syncthreads();
    }
  }
}

// Cluster offsets and the chunk list: cluster c owns sorted positions
// [coff[c], coff[c+1]) split into chunks cstart[c] .. cstart[c+1]-1; coff[k]
// is where the points without a valid center begin (n when there are none).
__global__ __launch_bounds__(1024) void k_chunk_list(const int* bbase, int nbs, int k, int n,
                                                     int* coff, int* cstart) {
  __shared__ long long sh[17];
  const int R = (k + 1023) / 1024;
  const int lo = min(k, (int)threadIdx.x * R), hi = min(k, lo + R);
  long long s = 0;
  for (int c = lo; c < hi; ++c) {
    const int o = bbase[(int64_t)c * nbs];
    const int o1 = bbase[(int64_t)(c + 1) * nbs];
    coff[c] = o;
    s += (o1 - o + kSegChunk - 1) / kSegChunk;
  }
  long long tot;
  long long run = block_excl_scan<long long, 1024>(s, sh, &tot);
  for (int c = lo; c < hi; ++c) {
    const int o = bbase[(int64_t)c * nbs];
    const int o1 = bbase[(int64_t)(c + 1) * nbs];
    cstart[c] = (int)run;
    run += (o1 - o + kSegChunk - 1) / kSegChunk;
  }
  if (threadIdx.x == 0) {
    coff[k] = bbase[(int64_t)k * nbs];
    cstart[k] = (int)tot;
  }
}


// Block q sums chunk q of its cluster: 256 threads form 256 / DW slices of DW
// lanes (lane = element), slice s owns the s-th of that many consecutive
// pieces of the chunk and adds its rows in point order, kSegAhead rows' loads
// issued ahead of their adds; the slices' sums are then added in slice order.
template <typename T>
__global__ __launch_bounds__(256) void k_seg_sum(const T* X, const float* row_scale, int d,
                                                 const int* sorted, const int* coff,
                                                 const int* cstart, int k, double* part) {
  __shared__ double red[256];
  const int q = blockIdx.x;
  if (q >= cstart[k]) return;
  int lo = 0, hi = k;  // largest c with cstart[c] <= q
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (cstart[mid] <= q) lo = mid; else hi = mid;
  }
  const int c = lo;
  const int p0 = coff[c] + (q - cstart[c]) * kSegChunk;
  const int p1 = min(coff[c + 1], p0 + kSegChunk);
  const int DW = seg_width(d), NS = 256 / DW;
  const int t = threadIdx.x, sl = t / DW, el = t % DW;
  const int len = p1 - p0, per = (len + NS - 1) / NS;
  const int a = p0 + min(len, sl * per), b = p0 + min(len, (sl + 1) * per);
  for (int e0 = 0; e0 < d; e0 += DW) {
    const int e = e0 + el;
    double acc = 0.0;
    if (e < d) {
      int p = a;
      for (; p + kSegAhead <= b; p += kSegAhead) {
        int idx[kSegAhead];
        float v[kSegAhead];
#pragma unroll
        for (int u = 0; u < kSegAhead; ++u) idx[u] = sorted[p + u];
#pragma unroll
        for (int u = 0; u < kSegAhead; ++u)
          v[u] = Elem<T>::get(X, (int64_t)idx[u] * d + e, row_scale_of<T>(row_scale, idx[u]));
#pragma unroll
        for (int u = 0; u < kSegAhead; ++u) acc += (double)v[u];
      }
      for (; p < b; ++p) {
        const int i = sorted[p];
        acc += (double)Elem<T>::get(X, (int64_t)i * d + e, row_scale_of<T>(row_scale, i));
      }
    }
    red[t] = acc;
    __syncthreads();
    if (t < DW && e0 + t < d) {
      double sum = 0.0;
      for (int j = 0; j < NS; ++j) sum += red[j * DW + t];
      part[(int64_t)q * d + e0 + t] = sum;
    }
    __syncthreads();
  }
}

// Block c divides cluster c: 256 threads form 256 / DW slices of DW lanes
// (lane = element); slice s adds the s-th of that many consecutive pieces of
// the cluster's chunk sums in chunk order, eight loads issued ahead of their
// adds; the slices' sums are then added in slice order.  A cluster of a
// million points has about 500 chunk sums, which one chain would add one
// batch of loads at a time.
__global__ __launch_bounds__(256) void k_centroid(const double* part, const int* coff,
                                                  const int* cstart, int d, float* C) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const int cnt = coff[c + 1] - coff[c];
  if (cnt == 0) return;  // an empty cluster keeps its center
  const int q0 = cstart[c], q1 = cstart[c + 1];
  const int DW = seg_width(d), NS = 256 / DW;
  const int t = threadIdx.x, sl = t / DW, el = t % DW;
  const int len = q1 - q0, per = (len + NS - 1) / NS;
  const int a = q0 + min(len, sl * per), b = q0 + min(len, (sl + 1) * per);
  for (int e0 = 0; e0 < d; e0 += DW) {
    const int e = e0 + el;
    double s = 0.0;
    if (e < d) {
      int q = a;
      for (; q + 8 <= b; q += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(q + u) * d + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
      for (; q < b; ++q) s += part[(int64_t)q * d + e];
    }
    red[t] = s;
    __syncthreads();
    if (t < DW && e0 + t < d) {
      double sum = 0.0;
      for (int j = 0; j < NS; ++j) sum += red[j * DW + t];
      C[(int64_t)c * d + e0 + t] = (float)(sum / (double)cnt);
    }
    __syncthreads();
  }
}

hipError_t launch_lloyd_update(kmpar_dtype dt, const void* X, const float* row_scale, int n, int d,
                               const int* A, int k, float* C, const LloydWs& w, hipStream_t s) {
  const int nbs = (n + kSortChunk - 1) / kSortChunk;
  const int64_t L = (int64_t)(k + 1) * nbs;  // keys 0 .. k
  const int ntiles = (int)((L + kScanTile - 1) / kScanTile);
  const size_t lds = (size_t)(k + 1) * sizeof(int);
  hipError_t e = hipFuncSetAttribute((const void*)k_sort_count,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_sort_scatter, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_count, dim3(nbs), dim3(256), lds, s, A, n, k, w.bcnt, nbs);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, w.bcnt, L, w.scan_tmp);
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, s, w.scan_tmp, ntiles, (int*)nullptr,
                     (int*)nullptr, 0, 0, (kmpar_stats*)nullptr);
  hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(256), 0, s, w.bcnt, L, w.scan_tmp);
  const int nbits = 32 - __builtin_clz((unsigned)k);  // bits of the largest key, k
  hipLaunchKernelGGL(k_sort_scatter, dim3(nbs), dim3(64), lds, s, A, n, k, nbits, w.bcnt, nbs,
                     w.sorted);
  hipLaunchKernelGGL(k_chunk_list, dim3(1), dim3(1024), 0, s, w.bcnt, nbs, k, n, w.coff, w.cstart);
  const int max_chunks = (n + kSegChunk - 1) / kSegChunk + k;
  switch (dt) {
    case KMPAR_F32:
      hipLaunchKernelGGL(k_seg_sum<float>, dim3(max_chunks), dim3(256), 0, s, (const float*)X,
                         row_scale, d, w.sorted, w.coff, w.cstart, k, w.part);
      break;
    case KMPAR_BF16:
      hipLaunchKernelGGL(k_seg_sum<bf16_t>, dim3(max_chunks), dim3(256), 0, s, (const bf16_t*)X,
                         row_scale, d, w.sorted, w.coff, w.cstart, k, w.part);
      break;
    case KMPAR_FP8_E4M3:
      hipLaunchKernelGGL(k_seg_sum<fp8_t>, dim3(max_chunks), dim3(256), 0, s, (const fp8_t*)X,
                         row_scale, d, w.sorted, w.coff, w.cstart, k, w.part);
      break;
  }
  hipLaunchKernelGGL(k_centroid, dim3(k), dim3(256), 0, s, w.part, w.coff, w.cstart, d, C);
  KMPAR_RET_LAST();
}

}  // namespace kmpar
