// The passes of k-means|| around the distance fold: first center, cost phi,
// Bernoulli draws with order-preserving compaction, candidate gather, the
// Step-7 weight histogram, the Step-8 weighted k-means++ recluster and the
// Lloyd centroid update.  Every reduction and scan runs in a fixed order, so
// results are bit-reproducible.
#include <math.h>

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
// Algorithm 2 step 4: point i is kept in round t iff u < p with
// p = min(1, ell * D2_i / phi) and u = U(seed, ROUND, (i, t, inst)).
__device__ __forceinline__ int keep_point(const float* D2, int i, double phi, double ell,
                                          uint64_t seed, int t, uint64_t inst) {
  if (!(phi > 0.0)) return 0;
  double p = ell * (double)D2[i] / phi;
  if (p > 1.0) p = 1.0;
  const double u = philox_uniform(seed, kTagRound, (uint64_t)i, (uint64_t)t, inst);
  return u < p ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_draw_count(const float* D2, int n, const double* phi,
                                                    double ell, uint64_t seed, int t,
                                                    uint64_t inst, int* cnt) {
  __shared__ int sh[8];
  const double ph = *phi;
  const int base = blockIdx.x * kDrawChunk;
  int c = 0;
#pragma unroll
  for (int r = 0; r < kDrawChunk / 256; ++r) {
    const int i = base + r * 256 + threadIdx.x;
    if (i < n) c += keep_point(D2, i, ph, ell, seed, t, inst);
  }
  const int tot = block_sum<int, 256>(c, sh);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

// In-place exclusive scan of a[0..L) by one block; *total = sum.
__global__ __launch_bounds__(1024) void k_scan1(int* a, int L, int* total) {
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
}

// Commits round t: m_t = min(total, cap), rs[t+1] = rs[t] + m_t.
__global__ void k_round_commit(const int* total, int* rs, int t, int cap, kmpar_stats* st) {
  if (threadIdx.x != 0) return;
  const int tot = *total;
  const int m = tot < cap ? tot : cap;
  rs[t + 1] = rs[t] + m;
  st->round_count[t] = m;
  if (tot > cap) st->status = KMPAR_E_OVERFLOW;
}

// Writes the kept point indices in increasing point order.
__global__ __launch_bounds__(256) void k_draw_write(const float* D2, int n, const double* phi,
                                                    double ell, uint64_t seed, int t,
                                                    uint64_t inst, const int* off, const int* rs,
                                                    int cap, int* cand_point) {
  __shared__ int sh[8];
  const double ph = *phi;
  const int base = blockIdx.x * kDrawChunk;
  int run = off[blockIdx.x];
  const int start = rs[t];
  for (int r = 0; r < kDrawChunk / 256; ++r) {
    const int i = base + r * 256 + threadIdx.x;
    const int keep = (i < n) ? keep_point(D2, i, ph, ell, seed, t, inst) : 0;
    int tot;
    const int rank = block_excl_scan<int, 256>(keep, sh, &tot);
    if (keep && run + rank < cap) cand_point[start + run + rank] = i;
    run += tot;
  }
}

hipError_t launch_draw(const float* D2, int n, const double* phi, double ell, uint64_t seed, int t,
                       uint64_t inst, int* cnt, int* scan_total, int* rs, int cap_round,
                       int* cand_point, kmpar_stats* st, hipStream_t s) {
  const int nb = (n + kDrawChunk - 1) / kDrawChunk;
  hipLaunchKernelGGL(k_draw_count, dim3(nb), dim3(256), 0, s, D2, n, phi, ell, seed, t, inst, cnt);
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, s, cnt, nb, scan_total);
  hipLaunchKernelGGL(k_round_commit, dim3(1), dim3(64), 0, s, scan_total, rs, t, cap_round, st);
  hipLaunchKernelGGL(k_draw_write, dim3(nb), dim3(256), 0, s, D2, n, phi, ell, seed, t, inst, cnt,
                     rs, cap_round, cand_point);
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
// atomics (exact, so the result does not depend on their order).
__global__ __launch_bounds__(256) void k_hist_lds(const int* A, int n, int* w, int nbins) {
  extern __shared__ int h[];
  for (int b = threadIdx.x; b < nbins; b += 256) h[b] = 0;
  __syncthreads();
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
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

constexpr int kLdsBudget = 64 * 1024;

hipError_t launch_hist(const int* A, int n, int* w, int nbins, hipStream_t s) {
  hipError_t e = launch_fill_i32(w, 0, nbins, s);
  if (e != hipSuccess) return e;
  const int blocks = 512;
  if ((size_t)nbins * 4 <= (size_t)kLdsBudget) {
    hipLaunchKernelGGL(k_hist_lds, dim3(blocks), dim3(256), (size_t)nbins * 4, s, A, n, w, nbins);
  } else {
    hipLaunchKernelGGL(k_hist_global, dim3(blocks), dim3(256), 0, s, A, n, w, nbins);
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
// Per pick: each block folds the previous pick into its E and publishes its
// FP64 partial; grid barrier; every block derives the same block bounds from
// the partials in block order; the block holding u*T finds the pick and
// publishes it; grid barrier.  Barriers are agent-scope release/acquire
// counters; a spin limit guarantees every wave exits (status KMPAR_E_HIP).
constexpr int kReclBlock = 256;
constexpr unsigned kSpinLimit = 1u << 22;
constexpr size_t kReclLdsBudget = 120 * 1024;

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned target, int* failed) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        *failed = 1;
        break;
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void store_f64(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_f64(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
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
  int slice_cap;       // LDS slice capacity (candidates per block)
  double* part;        // [2][G] block partials
  float* prow;         // [2][DP] row of the latest pick, published through memory
  unsigned* bar;       // barrier counter, zero on entry
  int* picks;          // [k] output: candidate ids
  float* centers;      // [k][d] output rows
  kmpar_stats* st;
};

__global__ __launch_bounds__(kReclBlock) void k_recluster_grid(ReclArgs a) {
  extern __shared__ float lds[];
  __shared__ double shd[kReclBlock / kWave + 1];
  __shared__ double runb[kReclBlock + 1];
  __shared__ double blockb[2];
  __shared__ double gpart[kReclMaxBlocks];
  __shared__ double sh_T;
  __shared__ int sh_pick, sh_owner, sh_failed, sh_stop;
  const int G = gridDim.x, b = blockIdx.x, tid = threadIdx.x, DP = a.DP, d = a.d;
  const int m = *a.rs_end;
  const int lo = (int)((int64_t)b * m / G), hi = (int)((int64_t)(b + 1) * m / G);
  const int ns = hi - lo;
  float* rows = lds;                                   // [slice_cap][DP]
  float* E = rows + (size_t)a.slice_cap * DP;          // [slice_cap]
  int* wl = reinterpret_cast<int*>(E + a.slice_cap);   // [slice_cap]
  float* cp = reinterpret_cast<float*>(wl + a.slice_cap);  // [DP]
  if (tid == 0) {
    sh_failed = 0;
    sh_stop = 0;
  }
  for (int idx = tid; idx < ns * DP; idx += kReclBlock) rows[idx] = a.Call[(int64_t)lo * DP + idx];
  for (int j = tid; j < ns; j += kReclBlock) wl[j] = a.w[lo + j];
  __syncthreads();
  // contiguous thread runs inside the slice, for the running sums
  const int R = (ns + kReclBlock - 1) / kReclBlock;
  const int rlo = min(ns, tid * R), rhi = min(ns, rlo + R);
  unsigned nbar = 0;
  int made = 0;
  for (int s = 0; s < a.k; ++s) {
    if (s > 0) {
      for (int e = tid; e < DP; e += kReclBlock)
        cp[e] = __uint_as_float(__hip_atomic_load(
            reinterpret_cast<const unsigned*>(&a.prow[((s - 1) & 1) * DP + e]), __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT));
      __syncthreads();
      for (int j = tid; j < ns; j += kReclBlock) {
        const float* r = rows + (size_t)j * DP;
        float acc = 0.0f;
        for (int e = 0; e < d; ++e) {
          const float t = r[e] - cp[e];
          acc = fmaf(t, t, acc);
        }
        E[j] = (s == 1) ? acc : fminf(E[j], acc);
      }
      __syncthreads();
    }
    double loc = 0.0;
    for (int j = rlo; j < rhi; ++j) loc += (s == 0) ? (double)wl[j] : (double)wl[j] * (double)E[j];
    double tot;
    const double ex = block_excl_scan<double, kReclBlock>(loc, shd, &tot);
    runb[tid] = ex;
    if (tid == 0) {
      runb[kReclBlock] = tot;
      store_f64(&a.part[(s & 1) * G + b], tot);
    }
    grid_barrier(a.bar, (++nbar) * (unsigned)G, &sh_failed);
    // every block: block bounds from the partials in block order (loaded in
    // parallel, summed in order by one thread)
    for (int q = tid; q < G; q += kReclBlock) gpart[q] = load_f64(&a.part[(s & 1) * G + q]);
    __syncthreads();
    if (tid == 0) {
      double run = 0.0, lo_b = 0.0, hi_b = 0.0;
      int owner = -1, last_pos = -1;
      double T = 0.0;
      for (int q = 0; q < G; ++q) T += gpart[q];
      sh_T = T;
      const double u = philox_uniform(a.seed, kTagRecluster, (uint64_t)s, 0, a.inst);
      const double thr = u * T;
      for (int q = 0; q < G; ++q) {
        const double v = gpart[q];
        const double nxt = (q + 1 < G) ? run + v : T;
        if (v > 0.0) last_pos = q;
        if (owner < 0 && run <= thr && thr < nxt && v > 0.0) {
          owner = q;
          lo_b = run;
          hi_b = nxt;
        }
        run += v;
      }
      if (!(T > 0.0) || sh_failed) {
        sh_stop = 1;
      } else if (owner < 0) {  // thr at or past the total by rounding
        owner = last_pos;
        lo_b = hi_b = INFINITY;
      }
      sh_owner = owner;
      blockb[0] = lo_b;
      blockb[1] = hi_b;
      sh_pick = 0x7fffffff;
    }
    __syncthreads();
    if (sh_stop) break;
    if (sh_owner == b) {
      const double u = philox_uniform(a.seed, kTagRecluster, (uint64_t)s, 0, a.inst);
      const double thr = u * sh_T;
      const double base = blockb[0];
      const double b0 = base + runb[tid];
      const double b1 = (tid + 1 < kReclBlock) ? base + runb[tid + 1] : blockb[1];
      if (isinf(base)) {
        // rounding fallback: the last candidate with positive mass
        if (tid == 0) {
          for (int j = ns - 1; j >= 0; --j) {
            const double v = (s == 0) ? (double)wl[j] : (double)wl[j] * (double)E[j];
            if (v > 0.0) {
              sh_pick = j;
              break;
            }
          }
        }
      } else if (b0 <= thr && thr < b1) {
        double run = b0;
        int pick = -1, last = -1;
        for (int j = rlo; j < rhi; ++j) {
          const double v = (s == 0) ? (double)wl[j] : (double)wl[j] * (double)E[j];
          run += v;
          if (v > 0.0) last = j;
          if (v > 0.0 && run > thr) {
            pick = j;
            break;
          }
        }
        if (pick < 0) pick = last;
        if (pick >= 0) atomicMin(&sh_pick, pick);
      }
      __syncthreads();
      if (sh_pick == 0x7fffffff) {
        // Thread-run bounds and the block bound come from different FP64
        // association orders; if no run claimed u*T, walk the slice in order.
        if (tid == 0) {
          double run = base;
          int last = -1;
          for (int j = 0; j < ns; ++j) {
            const double v = (s == 0) ? (double)wl[j] : (double)wl[j] * (double)E[j];
            run += v;
            if (v > 0.0) last = j;
            if (v > 0.0 && run > thr) {
              sh_pick = j;
              break;
            }
          }
          if (sh_pick == 0x7fffffff) sh_pick = last;
        }
        __syncthreads();
      }
      const int jl = sh_pick;
      for (int e = tid; e < d; e += kReclBlock) a.centers[(int64_t)s * d + e] = rows[(size_t)jl * DP + e];
      for (int e = tid; e < DP; e += kReclBlock)
        __hip_atomic_store(reinterpret_cast<unsigned*>(&a.prow[(s & 1) * DP + e]),
                           __float_as_uint(rows[(size_t)jl * DP + e]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      if (tid == 0) a.picks[s] = lo + jl;
    }
    grid_barrier(a.bar, (++nbar) * (unsigned)G, &sh_failed);
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
                                                          int cap_lds) {
  extern __shared__ float lds[];
  recluster_block<1024>(CallT, ldT, d, w, *rs_end, k, seed, inst, picks, centers, st, lds, cap_lds);
}

size_t recluster_block_lds(int capT, int k) { return (size_t)capT * 8 + (size_t)k * 8; }

hipError_t launch_recluster_block(const float* CallT, int capT, int d, const int* w,
                                  const int* rs_end, int k, uint64_t seed, uint64_t inst,
                                  int* picks, float* centers, kmpar_stats* st, hipStream_t s) {
  const size_t lds = recluster_block_lds(capT, k);
  hipError_t e = hipFuncSetAttribute((const void*)k_recluster_block,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_recluster_block, dim3(1), dim3(1024), lds, s, CallT, capT, d, w, rs_end, k,
                     seed, inst, picks, centers, st, capT);
  KMPAR_RET_LAST();
}

int recluster_blocks(int capT, int DP, int num_cu) {
  // Slices of about 512 candidates (a grid barrier costs ~0.8 us at 8-16
  // workgroups and grows with their number); each slice must fit the LDS budget.
  const size_t per = (size_t)DP * 4 + 8;
  int G = (capT + 511) / 512;
  const int min_g = (int)((capT * per + kReclLdsBudget - 1) / kReclLdsBudget);
  if (G < min_g) G = min_g;
  if (G > num_cu) G = num_cu;
  if (G > kReclMaxBlocks) G = kReclMaxBlocks;
  if (G < 1) G = 1;
  return G;
}

size_t recluster_lds(int capT, int DP, int G) {
  const int slice = (capT + G - 1) / G + 1;
  return (size_t)slice * ((size_t)DP * 4 + 8) + (size_t)DP * 4;
}

hipError_t launch_recluster(const float* Call, int DP, int capT, int d, const int* w,
                            const int* rs_end, int k, uint64_t seed, uint64_t inst, int G,
                            double* part, float* prow, unsigned* bar, int* picks, float* centers,
                            kmpar_stats* st, hipStream_t s) {
  hipError_t e = launch_fill_i32(reinterpret_cast<int*>(bar), 0, 1, s);
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
  a.slice_cap = (capT + G - 1) / G + 1;
  a.part = part;
  a.prow = prow;
  a.bar = bar;
  a.picks = picks;
  a.centers = centers;
  a.st = st;
  const size_t lds = recluster_lds(capT, DP, G);
  e = hipFuncSetAttribute((const void*)k_recluster_grid, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_recluster_grid, dim3(G), dim3(kReclBlock), lds, s, a);
  KMPAR_RET_LAST();
}

// ------------------------------------------------------------- Lloyd update
// Deterministic centroid update (Section 3.1 centroid; Section 1 Lloyd):
//  1. per-block cluster counts   bcnt[c * nbs + b]
//  2. exclusive scan of the flattened table -> each (cluster, block) slot
//  3. stable scatter of point indices into cluster-sorted order
//  4. cluster chunks of kSegChunk sorted points, summed in FP64 in order
//  5. per cluster: sum of its chunk sums in order, divided by the count.
__global__ __launch_bounds__(256) void k_sort_count(const int* A, int n, int k, int* bcnt,
                                                    int nbs) {
  extern __shared__ int h[];
  for (int c = threadIdx.x; c < k; c += 256) h[c] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortChunk;
  for (int r = threadIdx.x; r < kSortChunk; r += 256) {
    const int i = base + r;
    if (i < n) {
      const int a = A[i];
      if (a >= 0 && a < k) atomicAdd(&h[a], 1);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += 256) bcnt[(int64_t)c * nbs + blockIdx.x] = h[c];
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

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x % kWave;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// One wave per block scatters its chunk in point order; equal keys inside a
// 64-point tile are ranked by lane, and the per-cluster cursor advances once
// per key group.
__global__ __launch_bounds__(64) void k_sort_scatter(const int* A, int n, int k, const int* bbase,
                                                     int nbs, int* sorted) {
  extern __shared__ int cur[];
  for (int c = threadIdx.x; c < k; c += 64) cur[c] = bbase[(int64_t)c * nbs + blockIdx.x];
  __syncthreads();
  const int lane = threadIdx.x;
  const int base = blockIdx.x * kSortChunk;
  for (int tile = 0; tile < kSortChunk; tile += 64) {
    const int i = base + tile + lane;
    const int key0 = (i < n) ? A[i] : -1;
    const bool valid = key0 >= 0 && key0 < k;
    const int key = valid ? key0 : -1;
    uint64_t pending = __ballot(valid);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const int lkey = __shfl(key, leader, kWave);
      const uint64_t grp = __ballot(valid && key == lkey);
      const int pos0 = cur[lkey];
      if (valid && key == lkey) sorted[pos0 + __popcll(grp & lanemask_lt())] = i;
      __syncthreads();
      if (lane == leader) cur[lkey] = pos0 + __popcll(grp);
      __syncthreads();
      pending &= ~grp;
    }
  }
}

// Cluster offsets and the chunk list: cluster c owns sorted positions
// [coff[c], coff[c+1]) split into chunks cstart[c] .. cstart[c+1]-1.
__global__ __launch_bounds__(1024) void k_chunk_list(const int* bbase, int nbs, int k, int n,
                                                     int* coff, int* cstart) {
  __shared__ long long sh[17];
  const int R = (k + 1023) / 1024;
  const int lo = min(k, (int)threadIdx.x * R), hi = min(k, lo + R);
  long long s = 0;
  for (int c = lo; c < hi; ++c) {
    const int o = bbase[(int64_t)c * nbs];
    const int o1 = (c + 1 < k) ? bbase[(int64_t)(c + 1) * nbs] : n;
    coff[c] = o;
    s += (o1 - o + kSegChunk - 1) / kSegChunk;
  }
  long long tot;
  long long run = block_excl_scan<long long, 1024>(s, sh, &tot);
  for (int c = lo; c < hi; ++c) {
    const int o = bbase[(int64_t)c * nbs];
    const int o1 = (c + 1 < k) ? bbase[(int64_t)(c + 1) * nbs] : n;
    cstart[c] = (int)run;
    run += (o1 - o + kSegChunk - 1) / kSegChunk;
  }
  if (threadIdx.x == 0) {
    coff[k] = n;
    cstart[k] = (int)tot;
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_seg_sum(const T* X, const float* row_scale, int d,
                                                const int* sorted, const int* coff,
                                                const int* cstart, int k, double* part) {
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
  for (int e = threadIdx.x; e < d; e += 64) {
    double acc = 0.0;
    for (int p = p0; p < p1; ++p) {
      const int i = sorted[p];
      acc += (double)Elem<T>::get(X, (int64_t)i * d + e, row_scale_of<T>(row_scale, i));
    }
    part[(int64_t)q * d + e] = acc;
  }
}

__global__ __launch_bounds__(64) void k_centroid(const double* part, const int* coff,
                                                 const int* cstart, int d, float* C) {
  const int c = blockIdx.x;
  const int cnt = coff[c + 1] - coff[c];
  if (cnt == 0) return;  // an empty cluster keeps its center
  for (int e = threadIdx.x; e < d; e += 64) {
    double s = 0.0;
    for (int q = cstart[c]; q < cstart[c + 1]; ++q) s += part[(int64_t)q * d + e];
    C[(int64_t)c * d + e] = (float)(s / (double)cnt);
  }
}

hipError_t launch_lloyd_update(kmpar_dtype dt, const void* X, const float* row_scale, int n, int d,
                               const int* A, int k, float* C, const LloydWs& w, hipStream_t s) {
  const int nbs = (n + kSortChunk - 1) / kSortChunk;
  const int64_t L = (int64_t)k * nbs;
  const int ntiles = (int)((L + kScanTile - 1) / kScanTile);
  const size_t lds = (size_t)k * sizeof(int);
  hipLaunchKernelGGL(k_sort_count, dim3(nbs), dim3(256), lds, s, A, n, k, w.bcnt, nbs);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, w.bcnt, L, w.scan_tmp);
  hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, s, w.scan_tmp, ntiles, (int*)nullptr);
  hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(256), 0, s, w.bcnt, L, w.scan_tmp);
  hipLaunchKernelGGL(k_sort_scatter, dim3(nbs), dim3(64), lds, s, A, n, k, w.bcnt, nbs, w.sorted);
  hipLaunchKernelGGL(k_chunk_list, dim3(1), dim3(1024), 0, s, w.bcnt, nbs, k, n, w.coff, w.cstart);
  const int max_chunks = (n + kSegChunk - 1) / kSegChunk + k;
  switch (dt) {
    case KMPAR_F32:
      hipLaunchKernelGGL(k_seg_sum<float>, dim3(max_chunks), dim3(64), 0, s, (const float*)X,
                         row_scale, d, w.sorted, w.coff, w.cstart, k, w.part);
      break;
    case KMPAR_BF16:
      hipLaunchKernelGGL(k_seg_sum<bf16_t>, dim3(max_chunks), dim3(64), 0, s, (const bf16_t*)X,
                         row_scale, d, w.sorted, w.coff, w.cstart, k, w.part);
      break;
    case KMPAR_FP8_E4M3:
      hipLaunchKernelGGL(k_seg_sum<fp8_t>, dim3(max_chunks), dim3(64), 0, s, (const fp8_t*)X,
                         row_scale, d, w.sorted, w.coff, w.cstart, k, w.part);
      break;
  }
  hipLaunchKernelGGL(k_centroid, dim3(k), dim3(64), 0, s, w.part, w.coff, w.cstart, d, C);
  KMPAR_RET_LAST();
}

}  // namespace kmpar
