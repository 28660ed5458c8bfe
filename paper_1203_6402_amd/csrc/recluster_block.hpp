// Weighted k-means++ recluster (Algorithm 2 step 8 with Algorithm 1) in one
// workgroup: shared by the batched path (one workgroup per instance) and the
// single-instance path when the candidates' E and nearest-pick ids fit LDS.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace kmpar {

// Pick 0 has probability w_j / sum w (integer sums, exact in FP64); pick
// s >= 1 has probability w_j E_j / T, E_j the FP32 direct-form distance to
// the nearest earlier pick, every sum in FP64.  Pick s takes the smallest j
// whose running sum (thread runs, then candidate order) exceeds u*T with
// u = U(seed, RECL, (s, 0, inst)).  E_j and the nearest pick a_j live in LDS.
// A candidate's row is read only when the new pick can improve it: with
// D_pa = ||c_pick - c_a(j)||^2, the triangle inequality gives
// ||c_j - c_pick|| >= sqrt(D_pa) - sqrt(E_j), so D_pa > 4 E_j (1 + eps)
// implies ||c_j - c_pick||^2 > E_j and E_j cannot change (eps covers the
// FP32 rounding of both distances), so pruning leaves every E_j as the
// unpruned update would.
// Candidate rows are read from the dim-major copy CallT[e * ldT + j], so the
// lanes of a wave, which take consecutive candidates, read consecutive words.

// FP32 direct form sum_e (c_e - p_e)^2, e ascending, of dim-major column j
// against the row p: sixteen loads are issued before their sixteen fmas, so
// a thread waits for memory once per sixteen elements, not once per element.
__device__ __forceinline__ float col_dist(const float* __restrict__ CallT, int ldT, int j,
                                          const float* p, int d) {
  float acc = 0.0f;
  for (int e0 = 0; e0 < d; e0 += 16) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      v[u] = e0 + u < d ? CallT[(int64_t)(e0 + u) * ldT + j] : 0.0f;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (e0 + u < d) {
        const float t = v[u] - p[e0 + u];
        acc = fmaf(t, t, acc);
      }
    }
  }
  return acc;
}

template <int BS>
__device__ void recluster_block(const float* __restrict__ CallT, int ldT, int d,
                                const int* __restrict__ w, int m, int k, uint64_t seed,
                                uint64_t inst, int* picks, float* centers, kmpar_stats* st,
                                float* lds, int cap_lds, double band) {
  __shared__ double shd[BS / kWave + 1];
  __shared__ long long shl[BS / kWave + 1];
  __shared__ double bounds[BS + 1];
  __shared__ float cp[256];
  __shared__ int pick_sh, flag_sh;
  __shared__ double plo_sh, phi_sh;
  float* E = lds;                                        // [cap_lds]
  int* near = reinterpret_cast<int*>(lds + cap_lds);     // [cap_lds] pick number
  float* pd = reinterpret_cast<float*>(near + cap_lds);  // [k] D_pa of the current pick
  int* pk = reinterpret_cast<int*>(pd + k);              // [k] picks so far
  const float eps = 8.0f * (float)(d + 2) * 0x1.0p-24f;
  const int tid = threadIdx.x;
  const int R = (m + BS - 1) / BS;
  const int lo = min(m, tid * R), hi = min(m, lo + R);
  int made = 0;
  for (int s = 0; s < k; ++s) {
    const double u = philox_uniform(seed, kTagRecluster, (uint64_t)s, 0, inst);
    if (tid == 0) pick_sh = 0x7fffffff;
    double T;
    if (s == 0) {
      long long loc = 0;
      for (int j = lo; j < hi; ++j) loc += w[j];
      long long tot;
      const long long ex = block_excl_scan<long long, BS>(loc, shl, &tot);
      bounds[tid] = (double)ex;
      if (tid == 0) bounds[BS] = (double)tot;
      T = (double)tot;
    } else {
      double loc = 0.0;
      for (int j = lo; j < hi; ++j) loc += (double)w[j] * (double)E[j];
      double tot;
      const double ex = block_excl_scan<double, BS>(loc, shd, &tot);
      bounds[tid] = ex;
      if (tid == 0) bounds[BS] = tot;
      T = tot;
    }
    __syncthreads();
    if (!(T > 0.0)) break;
    const double thr = u * T;
    // The picked interval [lo, hi) of the running sums, recorded by the
    // thread that found the pick, decides whether u*T lay near enough to one
    // of its ends to have been decided the other way (pick_near_end; counted
    // in flagged_picks); a pick made by a rounding fallback always is.
    int my_pick = -1;
    double my_lo = 0.0, my_hi = 0.0;
    if (tid == 0) flag_sh = 0;
    if (bounds[tid] <= thr && thr < bounds[tid + 1]) {
      double run = bounds[tid];
      int pick = -1, last = -1;
      for (int j = lo; j < hi; ++j) {
        const double vv = (s == 0) ? (double)w[j] : (double)w[j] * (double)E[j];
        const double before = run;
        run += vv;
        if (vv > 0.0) last = j;
        if (vv > 0.0 && run > thr) {
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
      // Bounds of neighbouring runs come from different FP64 association
      // orders; should two runs claim u*T, the lower candidate id wins.
      atomicMin(&pick_sh, pick >= 0 ? pick : 0x7fffffff);
    }
    __syncthreads();
    if (my_pick >= 0 && my_pick == pick_sh) {
      plo_sh = my_lo;
      phi_sh = my_hi;
    }
    __syncthreads();
    if (pick_sh == 0x7fffffff) {
      // u*T at or past the total by rounding: the last candidate with mass.
      if (tid == 0) {
        pick_sh = -1;
        flag_sh = 1;
        for (int j = m - 1; j >= 0; --j) {
          const double vv = (s == 0) ? (double)w[j] : (double)w[j] * (double)E[j];
          if (vv > 0.0) {
            pick_sh = j;
            break;
          }
        }
      }
      __syncthreads();
    }
    const int pick = pick_sh;
    if (pick < 0) break;
    if (tid == 0 && (flag_sh || pick_near_end(thr, plo_sh, phi_sh, band))) st->flagged_picks += 1;
    for (int e = tid; e < d; e += BS) {
      const float x = CallT[(int64_t)e * ldT + pick];
      cp[e] = x;
      centers[(int64_t)s * d + e] = x;
    }
    if (tid == 0) {
      picks[s] = pick;  // written once per pick, never read back
      pk[s] = pick;
    }
    __syncthreads();
    for (int q = tid; q < s; q += BS) {
      pd[q] = col_dist(CallT, ldT, pk[q], cp, d);
    }
    __syncthreads();
    for (int j = tid; j < m; j += BS) {
      if (s > 0 && pd[near[j]] > 4.0f * E[j] * (1.0f + eps)) continue;
      const float acc = col_dist(CallT, ldT, j, cp, d);
      if (s == 0 || acc < E[j]) {
        E[j] = acc;
        near[j] = s;
      }
    }
    __syncthreads();
    made = s + 1;
  }
  if (tid == 0) {
    st->n_centers = made;
    if (made < k && st->status == KMPAR_OK) st->status = KMPAR_E_TOOFEW;
  }
}

}  // namespace kmpar
