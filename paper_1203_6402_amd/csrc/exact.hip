// D^2 sampling by an exponential race: the exact-ell rounds of k-means||
// (Section 5.3: exactly ell points per round, drawn in proportion to D^2
// without replacement) and k-means++ on all of X (Algorithm 1).
//
// Point i gets the clock key_i = -ln(V_i) / D^2_i, V_i uniform on (0, 1]
// from Philox tag 4 at counter (i, t, inst) (Efraimidis & Spirakis,
// "Weighted random sampling with a reservoir", IPL 2006): key_i is
// exponential with rate D^2_i, so the smallest key is one D^2 draw and the
// ell smallest are ell successive draws without replacement.  A point with
// D^2 = 0 gets +inf and is never drawn.  Keys are non-negative doubles, so
// their bit patterns order like unsigned integers; a radix select over
// those bits (eleven-bit digits, one histogram pass each) finds the ell-th
// smallest key tau exactly, and a round keeps the keys below tau and, among
// keys equal to tau, the lowest indices.  With ell = 1 and r = k - 1 the
// rounds make exactly the draws of k-means++.
#include <limits.h>
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "rows.hpp"

namespace kmpar {

constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;  // +inf: never drawn
constexpr int kRadixBins = 2048;
constexpr int kRadixLevels = 6;
// Level L of the select reads the digit of width radix_width(L) at bit
// radix_shift(L): bits 62 .. 52, 51 .. 41, ..., 18 .. 8, then 7 .. 0 (bit
// 63, the sign, is 0 for every key).
__host__ __device__ constexpr int radix_shift(int L) { return L < 5 ? 52 - 11 * L : 0; }
__host__ __device__ constexpr int radix_width(int L) { return L < 5 ? 11 : 8; }

// The race clock of point i in draw t.  0 - ln(V) is +0 when V = 1, so a
// key is never -0 (whose bits would sort above every positive key).
// -ln V of point i's race draw in round (step) t; the key is -ln V / D^2.
__device__ __forceinline__ double race_neglog(uint64_t seed, uint64_t i, uint64_t t, uint64_t inst) {
  const uint64_t w = philox_word0(seed, kTagExact, i, t, inst);
  const double v = (double)((w >> 11) + 1) * 0x1.0p-53;
  return 0.0 - log(v);
}
__device__ __forceinline__ double race_key_of(float d2, double neglog) {
  return d2 > 0.0f ? neglog / (double)d2 : INFINITY;
}
__device__ __forceinline__ double race_key(float d2, uint64_t seed, uint64_t i, uint64_t t,
                                           uint64_t inst) {
  if (!(d2 > 0.0f)) return INFINITY;
  return race_key_of(d2, race_neglog(seed, i, t, inst));
}

__device__ __forceinline__ unsigned long long key_bits(double k) {
  return (unsigned long long)__double_as_longlong(k);
}

// ----------------------------------------------------------- exact rounds
// Keys of round t and the histogram of their top digit (finite keys only).
__global__ __launch_bounds__(256) void k_exact_keys(const float* D2, int n, uint64_t seed, int t,
                                                    uint64_t inst, unsigned long long* keys,
                                                    int* hist) {
  __shared__ int h[kRadixBins];
  for (int b = threadIdx.x; b < kRadixBins; b += 256) h[b] = 0;
  __syncthreads();
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const unsigned long long b = key_bits(race_key(D2[i], seed, (uint64_t)i, (uint64_t)t, inst));
    keys[i] = b;
    if (b < kInfBits) atomicAdd(&h[(int)(b >> radix_shift(0))], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kRadixBins; b += 256)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Histogram of level L's digit over the keys inside the bucket chosen so far.
__global__ __launch_bounds__(256) void k_exact_hist(int L, const unsigned long long* keys, int n,
                                                    const ExactState* st, int* hist) {
  __shared__ int h[kRadixBins];
  if (st->m == 0) return;
  const unsigned long long prefix = st->prefix;
  const int sh = radix_shift(L), w = radix_width(L);
  const unsigned long long mask = (1ull << w) - 1;
  for (int b = threadIdx.x; b < kRadixBins; b += 256) h[b] = 0;
  __syncthreads();
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const unsigned long long b = keys[i];
    if (b < kInfBits && (b >> (sh + w)) == prefix) atomicAdd(&h[(int)((b >> sh) & mask)], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kRadixBins; b += 256)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// One block: at level 0 fixes m = min(ell, finite keys); at every level
// finds the digit whose bucket holds the need-th smallest remaining key and
// appends it to the prefix; clears the histogram for the next level.  After
// the last level the prefix is tau itself and tie_count / tie_need say how
// many keys equal tau and how many of them the round takes.
__global__ __launch_bounds__(256) void k_exact_pick(int L, int ell, int* hist, ExactState* st) {
  __shared__ int sh[256 / kWave + 1];
  constexpr int R = kRadixBins / 256;
  const int w = radix_width(L), nbins = 1 << w;
  int v[R];
  int loc = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int b = threadIdx.x * R + r;
    v[r] = b < nbins ? hist[b] : 0;
    loc += v[r];
  }
  int tot;
  const int ex = block_excl_scan<int, 256>(loc, sh, &tot);
  if (L == 0 && threadIdx.x == 0) {
    st->m = min(ell, tot);
    st->need = st->m;
    st->prefix = 0;
    st->tie_count = 0;
    st->tie_need = 0;
    st->tie_last = INT_MAX;
  }
  __syncthreads();
  const int m = st->m, need = st->need;
  const unsigned long long prefix = st->prefix;
  __syncthreads();
  if (m > 0 && ex < need && need <= ex + loc) {
    int run = ex;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (run < need && need <= run + v[r]) {
        st->prefix = (prefix << w) | (unsigned long long)(threadIdx.x * R + r);
        st->need = need - run;
        if (L == kRadixLevels - 1) {
          st->tie_count = v[r];
          st->tie_need = need - run;
        }
      }
      run += v[r];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int b = threadIdx.x * R + r;
    if (b < nbins) hist[b] = 0;
  }
}

// When only some of the keys equal to tau are taken: the index of the last
// one taken, walking the points in index order (one block; keys equal in
// all 64 bits are all but impossible, so this almost always returns at once).
__global__ __launch_bounds__(1024) void k_exact_ties(const unsigned long long* keys, int n,
                                                     ExactState* st) {
  __shared__ int sh[1024 / kWave + 1];
  if (st->m == 0 || st->tie_need >= st->tie_count) return;
  const unsigned long long tau = st->prefix;
  const int need = st->tie_need;
  int base = 0;
  for (int i0 = 0; i0 < n; i0 += 1024) {
    const int i = i0 + threadIdx.x;
    const int eq = (i < n && keys[i] == tau) ? 1 : 0;
    int tot;
    const int ex = block_excl_scan<int, 1024>(eq, sh, &tot);
    if (eq && base + ex + 1 == need) st->tie_last = i;
    base += tot;
    if (base >= need) break;
  }
}

// Keep masks and per-block counts of round t (the layout the compaction
// reads), and the count of keys within the relative band of tau: draws that
// the error of their D^2 could have moved across the threshold.
__global__ __launch_bounds__(256) void k_exact_count(const unsigned long long* keys, int n,
                                                     const ExactState* st, double band, int* cnt,
                                                     uint64_t* keep, kmpar_stats* stats) {
  __shared__ int sh[8];
  const int m = st->m;
  const unsigned long long tau = st->prefix;
  const int tie_last = st->tie_last;
  const double taud = __longlong_as_double((long long)tau);
  const int base = blockIdx.x * kDrawChunk;
  const int wv = threadIdx.x / kWave;
  int c = 0, nf = 0;
#pragma unroll
  for (int r = 0; r < kDrawChunk / 256; ++r) {
    const int i = base + r * 256 + threadIdx.x;
    int kp = 0;
    if (i < n && m > 0) {
      const unsigned long long b = keys[i];
      if (b < kInfBits) {
        kp = (b < tau || (b == tau && i <= tie_last)) ? 1 : 0;
        const double k = __longlong_as_double((long long)b);
        nf += (k <= taud * (1.0 + band) && k * (1.0 + band) >= taud) ? 1 : 0;
      }
    }
    c += kp;
    const uint64_t bal = __ballot(kp);
    if (threadIdx.x % kWave == 0) keep[(int64_t)blockIdx.x * (kDrawChunk / 64) + r * 4 + wv] = bal;
  }
  const int tot = block_sum<int, 256>(c, sh);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
  const int ftot = block_sum<int, 256>(nf, sh);
  if (threadIdx.x == 0 && ftot) atomicAdd(&stats->flagged_draws, ftot);
}

hipError_t launch_exact_round(const float* D2, int n, int ell, uint64_t seed, int t, uint64_t inst,
                              double band, const ExactWs& w, int* cnt, uint64_t* keep,
                              int* scan_total, int* rs, int cap_round, int* cand_point,
                              kmpar_stats* st, hipStream_t s) {
  const int grid = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_exact_keys, dim3(grid), dim3(256), 0, s, D2, n, seed, t, inst, w.keys,
                     w.hist);
  hipLaunchKernelGGL(k_exact_pick, dim3(1), dim3(256), 0, s, 0, ell, w.hist, w.state);
  for (int L = 1; L < kRadixLevels; ++L) {
    hipLaunchKernelGGL(k_exact_hist, dim3(grid), dim3(256), 0, s, L, w.keys, n, w.state, w.hist);
    hipLaunchKernelGGL(k_exact_pick, dim3(1), dim3(256), 0, s, L, ell, w.hist, w.state);
  }
  hipLaunchKernelGGL(k_exact_ties, dim3(1), dim3(1024), 0, s, w.keys, n, w.state);
  const int nb = (n + kDrawChunk - 1) / kDrawChunk;
  hipLaunchKernelGGL(k_exact_count, dim3(nb), dim3(256), 0, s, w.keys, n, w.state, band, cnt, keep,
                     st);
  return launch_round_compact(n, cnt, keep, scan_total, rs, t, cap_round, cand_point, st, s);
}

size_t exact_keys_bytes(int64_t n) { return (size_t)n * sizeof(unsigned long long); }
int exact_hist_bins() { return kRadixBins; }

// ------------------------------------------------------------- k-means++
// The first center: point Index(n) of the FIRST stream (as Algorithm 2 step
// 1 draws it), its row (decoded to FP32) into crow and centers[0].
template <typename T>
__global__ __launch_bounds__(256) void k_kpp_first(const T* X, const float* row_scale, int n, int d,
                                                   uint64_t seed, uint64_t inst, int* stop,
                                                   int* picks, float* centers, float* crow,
                                                   kmpar_stats* st) {
  __shared__ int sp;
  if (threadIdx.x == 0) {
    sp = (int)philox_index(seed, kTagFirst, 0, 0, inst, (uint64_t)n);
    picks[0] = sp;
    *stop = 0;
    st->round_count[0] = 1;
    st->status = KMPAR_OK;
    st->n_rescanned = 0;
    st->flagged_draws = 0;
    st->flagged_picks = 0;
  }
  __syncthreads();
  const int p = sp;
  const float sc = row_scale_of<T>(row_scale, p);
  for (int e = threadIdx.x; e < d; e += 256) {
    const float v = Elem<T>::get(X, (int64_t)p * d + e, sc);
    crow[e] = v;
    centers[e] = v;
  }
}

// One step over blocks of one wave and 64 rows: the rows, one contiguous
// span, are copied into LDS by direct 16-byte global-to-LDS loads (the one
// partial block at the end of X copies them lane by lane); each lane folds
// the latest center crow into its point's D^2 (FP32 direct form, coordinates
// in ascending order, as every fold computes it; first: D^2 is that
// distance), then, when t > 0, computes the key of draw t; the block writes
// its smallest (key, index) and the FP64 sum of its D^2 (fixed order).
typedef __attribute__((address_space(3))) void kpp_lds_void;
typedef const __attribute__((address_space(1))) void kpp_gbl_void;

template <typename T>
__global__ __launch_bounds__(64) void k_kpp_step(const T* X, const float* row_scale, int n, int d,
                                                 const float* crow, int first, uint64_t seed,
                                                 int t, uint64_t inst, const int* stop, float* D2,
                                                 unsigned long long* pkey, int* pidx,
                                                 double* pphi) {
  extern __shared__ __attribute__((aligned(16))) char rows[];  // [64][d] raw elements
  if (*stop) return;
  constexpr int S = (int)sizeof(T);
  const int lane = threadIdx.x, rowb = d * S;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int64_t i = p0 + lane;
  const bool live = i < n;
  if (p0 + 64 <= n) {
    const int bytes = 64 * rowb;  // a multiple of 16
    const char* src = reinterpret_cast<const char*>(X) + p0 * rowb;
    for (int v0 = 0; v0 < bytes; v0 += 1024)
      if (v0 + 16 * lane < bytes)
        __builtin_amdgcn_global_load_lds((kpp_gbl_void*)(src + v0 + 16 * lane),
                                         (kpp_lds_void*)(rows + v0), 16, 0, 0);
  } else if (live) {
    for (int e = 0; e < d; ++e) reinterpret_cast<T*>(rows)[lane * d + e] = X[i * d + e];
  }
  const float sc = live ? row_scale_of<T>(row_scale, i) : 1.0f;
  // the draw does not depend on the rows: computed while they are in flight
  const double nl = (live && t > 0) ? race_neglog(seed, (uint64_t)i, (uint64_t)t, inst) : 0.0;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  unsigned long long kb = ~0ull;
  int ki = INT_MAX;
  double ph = 0.0;
  if (live) {
    const T* xr = reinterpret_cast<const T*>(rows + lane * rowb);
    float acc = 0.0f;
    for (int e = 0; e < d; ++e) {
      const float tt = Elem<T>::get(xr, e, sc) - crow[e];
      acc = fmaf(tt, tt, acc);
    }
    float dd = acc;
    if (!first) {
      dd = D2[i];
      if (acc < dd) dd = acc;
    }
    D2[i] = dd;
    ph = (double)dd;
    if (t > 0) {
      kb = key_bits(race_key_of(dd, nl));
      ki = (int)i;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long ob = __shfl_xor(kb, off, kWave);
    const int oi = __shfl_xor(ki, off, kWave);
    if (ob < kb || (ob == kb && oi < ki)) {
      kb = ob;
      ki = oi;
    }
  }
  ph = wave_sum(ph);
  if (lane == 0) {
    pkey[blockIdx.x] = kb;
    pidx[blockIdx.x] = ki;
    pphi[blockIdx.x] = ph;
  }
}

// One block: the cost of the first s centers (FP64, the partials of
// k_kpp_reduce summed in a fixed order) into phi_steps[s - 1] (and psi when
// s = 1); for s < k the smallest (key, index) over them is center s, whose
// row goes to crow
// and centers[s].  An infinite smallest key (every point on a center) ends
// the run with KMPAR_E_TOOFEW.
template <typename T>
__global__ __launch_bounds__(1024) void k_kpp_pick(const unsigned long long* pkey, const int* pidx,
                                                   const double* pphi, int nb, const T* X,
                                                   const float* row_scale, int d, int s, int k,
                                                   int* stop, int* picks, float* centers,
                                                   float* crow, double* phi_steps,
                                                   kmpar_stats* st) {
  __shared__ unsigned long long skb[1024 / kWave];
  __shared__ int ski[1024 / kWave];
  __shared__ double sh[1024 / kWave + 1];
  __shared__ int sp;
  if (*stop) return;
  unsigned long long kb = ~0ull;
  int ki = INT_MAX;
  double ph = 0.0;
  // block partials b = tid, tid + 1024, ... (each wave's loads coalesced),
  // kPickAhead rounds of loads in flight before they are added in that order
  constexpr int kPickAhead = 8;
  for (int b0 = threadIdx.x; b0 < nb; b0 += kPickAhead * 1024) {
    double vp[kPickAhead];
    unsigned long long vk[kPickAhead];
    int vi[kPickAhead];
#pragma unroll
    for (int u = 0; u < kPickAhead; ++u) {
      const int b = b0 + u * 1024;
      vp[u] = b < nb ? pphi[b] : 0.0;
      vk[u] = b < nb ? pkey[b] : ~0ull;
      vi[u] = b < nb ? pidx[b] : INT_MAX;
    }
#pragma unroll
    for (int u = 0; u < kPickAhead; ++u) {
      if (b0 + u * 1024 < nb) ph += vp[u];
      if (vk[u] < kb || (vk[u] == kb && vi[u] < ki)) {
        kb = vk[u];
        ki = vi[u];
      }
    }
  }
  const double phi = block_sum<double, 1024>(ph, sh);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long ob = __shfl_xor(kb, off, kWave);
    const int oi = __shfl_xor(ki, off, kWave);
    if (ob < kb || (ob == kb && oi < ki)) {
      kb = ob;
      ki = oi;
    }
  }
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  if (lane == 0) {
    skb[wv] = kb;
    ski[wv] = ki;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 1024 / kWave; ++q)
      if (skb[q] < kb || (skb[q] == kb && ski[q] < ki)) {
        kb = skb[q];
        ki = ski[q];
      }
    if (phi_steps) phi_steps[s - 1] = phi;
    if (s == 1) st->phi[0] = phi;
    sp = -1;
    if (s >= k) {
      st->n_centers = k;
      st->n_candidates = k;
    } else if (kb >= kInfBits) {
      *stop = 1;
      st->n_centers = s;
      st->n_candidates = s;
      st->status = KMPAR_E_TOOFEW;
    } else {
      sp = ki;
      picks[s] = ki;
    }
  }
  __syncthreads();
  const int p = sp;
  if (p < 0) return;
  const float sc = row_scale_of<T>(row_scale, p);
  for (int e = threadIdx.x; e < d; e += 1024) {
    const float v = Elem<T>::get(X, (int64_t)p * d + e, sc);
    crow[e] = v;
    centers[(int64_t)s * d + e] = v;
  }
}

// First level of the pick: block q reduces the step's block partials
// [q per, (q + 1) per) to one (smallest key, its point, FP64 D^2 sum), in a
// fixed order; the pick then reduces these kKppQ partials.
__global__ __launch_bounds__(256) void k_kpp_reduce(const unsigned long long* pkey, const int* pidx,
                                                    const double* pphi, int nb, const int* stop,
                                                    unsigned long long* qkey, int* qidx,
                                                    double* qphi) {
  __shared__ double sh[256 / kWave + 1];
  __shared__ unsigned long long skb[256 / kWave];
  __shared__ int ski[256 / kWave];
  if (*stop) return;
  const int per = (nb + gridDim.x - 1) / gridDim.x;
  const int b0 = min(nb, (int)blockIdx.x * per), b1 = min(nb, b0 + per);
  unsigned long long kb = ~0ull;
  int ki = INT_MAX;
  double ph = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += 256) {
    ph += pphi[b];
    const unsigned long long k = pkey[b];
    const int i = pidx[b];
    if (k < kb || (k == kb && i < ki)) {
      kb = k;
      ki = i;
    }
  }
  const double tot = block_sum<double, 256>(ph, sh);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long ob = __shfl_xor(kb, off, kWave);
    const int oi = __shfl_xor(ki, off, kWave);
    if (ob < kb || (ob == kb && oi < ki)) {
      kb = ob;
      ki = oi;
    }
  }
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  if (lane == 0) {
    skb[wv] = kb;
    ski[wv] = ki;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 256 / kWave; ++q)
      if (skb[q] < kb || (skb[q] == kb && ski[q] < ki)) {
        kb = skb[q];
        ki = ski[q];
      }
    qkey[blockIdx.x] = kb;
    qidx[blockIdx.x] = ki;
    qphi[blockIdx.x] = tot;
  }
}

template <typename T>
static hipError_t run_kmeanspp(const void* Xv, const float* rsc, int n, int d, int k,
                               uint64_t seed, uint64_t inst, const KppWs& w, int* picks,
                               float* centers, double* phi_steps, kmpar_stats* st, hipStream_t s) {
  const T* X = static_cast<const T*>(Xv);
  const int nb = (n + 63) / 64;
  const size_t lds = (size_t)64 * d * sizeof(T);  // the block's raw rows
  hipError_t e = hipFuncSetAttribute((const void*)k_kpp_step<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kpp_first<T>, dim3(1), dim3(256), 0, s, X, rsc, n, d, seed, inst, w.stop,
                     picks, centers, w.crow, st);
  for (int step = 1; step <= k; ++step) {
    hipLaunchKernelGGL(k_kpp_step<T>, dim3(nb), dim3(64), lds, s, X, rsc, n, d, w.crow,
                       step == 1 ? 1 : 0, seed, step < k ? step : 0, inst, w.stop, w.D2, w.pkey,
                       w.pidx, w.pphi);
    hipLaunchKernelGGL(k_kpp_reduce, dim3(kKppQ), dim3(256), 0, s, w.pkey, w.pidx, w.pphi, nb,
                       w.stop, w.qkey, w.qidx, w.qphi);
    hipLaunchKernelGGL(k_kpp_pick<T>, dim3(1), dim3(1024), 0, s, w.qkey, w.qidx, w.qphi, kKppQ, X,
                       rsc, d, step, k, w.stop, picks, centers, w.crow, phi_steps, st);
  }
  return hipGetLastError();
}

hipError_t launch_kmeanspp(kmpar_dtype dt, const void* X, const float* rsc, int n, int d, int k,
                           uint64_t seed, uint64_t inst, const KppWs& w, int* picks,
                           float* centers, double* phi_steps, kmpar_stats* st, hipStream_t s) {
  switch (dt) {
    case KMPAR_F32:
      return run_kmeanspp<float>(X, rsc, n, d, k, seed, inst, w, picks, centers, phi_steps, st, s);
    case KMPAR_BF16:
      return run_kmeanspp<bf16_t>(X, rsc, n, d, k, seed, inst, w, picks, centers, phi_steps, st, s);
    case KMPAR_FP8_E4M3:
      return run_kmeanspp<fp8_t>(X, rsc, n, d, k, seed, inst, w, picks, centers, phi_steps, st, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------ Lloyd until stable
// Points whose assignment differs between two iterations, counted into *out.
__global__ __launch_bounds__(256) void k_count_changed(const int* a, const int* b, int n, int* out) {
  __shared__ int sh[8];
  int c = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) c += a[i] != b[i];
  const int tot = block_sum<int, 256>(c, sh);
  if (threadIdx.x == 0 && tot) atomicAdd(out, tot);
}

hipError_t launch_count_changed(const int* a, const int* b, int n, int* out, hipStream_t s) {
  hipError_t e = launch_fill_i32(out, 0, 1, s);
  if (e != hipSuccess) return e;
  const int grid = std::min((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_count_changed, dim3(grid), dim3(256), 0, s, a, b, n, out);
  return hipGetLastError();
}

}  // namespace kmpar
