// Batched k-means|| (Algorithm 2 for many independent instances at once).
//
// Every pass of the single-instance path becomes one grouped launch over all
// instances: a block finds its (instance, tile) by binary search in a
// prefix array that a planning kernel builds on the device from the
// instance table.  The distance pass is grouped by padded row length so it
// stays templated; the weighted k-means++ recluster runs one workgroup per
// instance and skips candidates that the new pick provably cannot improve.
#include <math.h>

#include <map>

#include "common.hpp"
#include "kernels.hpp"
#include "recluster_block.hpp"

namespace kmpar {

namespace {

constexpr int kBFold = 256;   // points per fold block
constexpr int kBRecl = 256;   // threads of a recluster workgroup

__host__ __device__ inline int64_t al256(int64_t v) { return (v + 255) / 256 * 256; }

// Sub-buffers of one instance's workspace region (byte offsets).
struct Region {
  int64_t D2, A, phi_part, cnt, rs, tot, cand, Call, CallT, w, picks, st, bytes;
  int64_t capT;
};

__host__ __device__ inline Region region_of(int64_t n, int d, int k, double ell, int rounds) {
  const int DP = padded_dim_hd(d);
  const int64_t capT = 1 + (int64_t)rounds * cap_round_hd(n, ell);
  Region r;
  int64_t o = 0;
  r.D2 = o;       o = al256(o + 4 * n);
  r.A = o;        o = al256(o + 4 * n);
  r.phi_part = o; o = al256(o + 8 * ((n + kPhiChunk - 1) / kPhiChunk));
  r.cnt = o;      o = al256(o + 4 * ((n + kDrawChunk - 1) / kDrawChunk + 1));
  r.rs = o;       o = al256(o + 4 * (rounds + 2));
  r.tot = o;      o = al256(o + 16);
  r.cand = o;     o = al256(o + 4 * capT);
  r.Call = o;     o = al256(o + 4 * capT * DP);
  r.CallT = o;    o = al256(o + 4 * capT * DP);
  r.capT = capT;
  r.w = o;        o = al256(o + 4 * capT);
  r.picks = o;    o = al256(o + 4 * k);
  r.st = o;       o = al256(o + (int64_t)sizeof(kmpar_stats));
  r.bytes = o;
  return r;
}

}  // namespace

// ------------------------------------------------------------------ layout
// Plan area at the start of the workspace:
//   off[count+1]        int64  instance region offsets (from the region base)
//   pre_draw[count+1]   int32  prefix of ceil(n/kDrawChunk)
//   pre_phi[count+1]    int32  prefix of ceil(n/kPhiChunk)
//   glist[count]        int32  instances ordered by fold group (stable)
//   gpre[count+G]       int32  per group, prefix of ceil(n/kBFold) tiles
//   gbeg[G+1]           int32  group g owns glist[gbeg[g] .. gbeg[g+1])
struct PlanPtrs {
  int64_t* off;
  int* pre_draw;
  int* pre_phi;
  int* glist;
  int* gpre;
  int* gbeg;
  char* regions;
};

static PlanPtrs plan_ptrs(void* ws, int count, int G) {
  char* b = static_cast<char*>(ws);
  int64_t o = 0;
  PlanPtrs p;
  p.off = reinterpret_cast<int64_t*>(b + o);  o = al256(o + 8 * (int64_t)(count + 1));
  p.pre_draw = reinterpret_cast<int*>(b + o); o = al256(o + 4 * (int64_t)(count + 1));
  p.pre_phi = reinterpret_cast<int*>(b + o);  o = al256(o + 4 * (int64_t)(count + 1));
  p.glist = reinterpret_cast<int*>(b + o);    o = al256(o + 4 * (int64_t)count);
  p.gpre = reinterpret_cast<int*>(b + o);     o = al256(o + 4 * (int64_t)(count + G));
  p.gbeg = reinterpret_cast<int*>(b + o);     o = al256(o + 4 * (int64_t)(G + 1));
  p.regions = b + o;
  return p;
}

struct GroupTable {
  int G;
  int dp[kBatchMaxGroups];
};

// One block of 1024 threads: region offsets, work-list prefixes, fold groups.
__global__ __launch_bounds__(1024) void kb_plan(const kmpar_instance* inst, int count, int rounds,
                                                GroupTable gt, PlanPtrs p) {
  __shared__ long long shl[17];
  const int R = (count + 1023) / 1024;
  const int lo = min(count, (int)threadIdx.x * R), hi = min(count, lo + R);
  long long s_bytes = 0, s_draw = 0, s_phi = 0;
  for (int i = lo; i < hi; ++i) {
    const kmpar_instance& I = inst[i];
    s_bytes += region_of(I.n, I.d, I.k, I.ell, rounds).bytes;
    s_draw += (I.n + kDrawChunk - 1) / kDrawChunk;
    s_phi += (I.n + kPhiChunk - 1) / kPhiChunk;
  }
  long long tb, td, tp;
  long long eb = block_excl_scan<long long, 1024>(s_bytes, shl, &tb);
  long long ed = block_excl_scan<long long, 1024>(s_draw, shl, &td);
  long long ep = block_excl_scan<long long, 1024>(s_phi, shl, &tp);
  for (int i = lo; i < hi; ++i) {
    const kmpar_instance& I = inst[i];
    p.off[i] = eb;
    p.pre_draw[i] = (int)ed;
    p.pre_phi[i] = (int)ep;
    eb += region_of(I.n, I.d, I.k, I.ell, rounds).bytes;
    ed += (I.n + kDrawChunk - 1) / kDrawChunk;
    ep += (I.n + kPhiChunk - 1) / kPhiChunk;
  }
  if (threadIdx.x == 0) {
    p.off[count] = tb;
    p.pre_draw[count] = (int)td;
    p.pre_phi[count] = (int)tp;
  }
  // fold groups: stable partition by padded dim, tile prefixes per group
  long long base = 0;
  for (int g = 0; g < gt.G; ++g) {
    long long c = 0, t = 0;
    for (int i = lo; i < hi; ++i)
      if (padded_dim_hd(inst[i].d) == gt.dp[g]) {
        c += 1;
        t += (inst[i].n + kBFold - 1) / kBFold;
      }
    long long tc, tt;
    long long ec = block_excl_scan<long long, 1024>(c, shl, &tc);
    long long et = block_excl_scan<long long, 1024>(t, shl, &tt);
    for (int i = lo; i < hi; ++i)
      if (padded_dim_hd(inst[i].d) == gt.dp[g]) {
        p.glist[base + ec] = i;
        p.gpre[base + g + ec] = (int)et;
        ec += 1;
        et += (inst[i].n + kBFold - 1) / kBFold;
      }
    if (threadIdx.x == 0) {
      p.gbeg[g] = (int)base;
      p.gpre[base + g + tc] = (int)tt;
    }
    base += tc;
    __syncthreads();
  }
  if (threadIdx.x == 0) p.gbeg[gt.G] = (int)base;
}

// Largest i in [0, len) with pre[i] <= v.
__device__ __forceinline__ int find_owner(const int* pre, int len, int v) {
  int lo = 0, hi = len;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

struct BView {
  const kmpar_instance* I;
  Region r;
  char* base;
  template <typename P>
  __device__ __forceinline__ P* at(int64_t off) const { return reinterpret_cast<P*>(base + off); }
};

__device__ __forceinline__ BView bview(const kmpar_instance* inst, int i, const PlanPtrs& p,
                                       int rounds) {
  BView v;
  v.I = inst + i;
  v.r = region_of(v.I->n, v.I->d, v.I->k, v.I->ell, rounds);
  v.base = p.regions + p.off[i];
  return v;
}

// ------------------------------------------------------------ first center
__global__ void kb_first(const kmpar_instance* inst, int count, int rounds, PlanPtrs p,
                         uint64_t seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const BView v = bview(inst, i, p, rounds);
  const int i0 = (int)philox_index(seed, kTagFirst, 0, 0, (uint64_t)i, (uint64_t)v.I->n);
  v.at<int>(v.r.cand)[0] = i0;
  int* rs = v.at<int>(v.r.rs);
  rs[0] = 0;
  rs[1] = 1;
  kmpar_stats* st = v.at<kmpar_stats>(v.r.st);
  st->round_count[0] = 1;
  st->status = KMPAR_OK;
  st->n_rescanned = 0;
  st->flagged_draws = 0;
  st->flagged_picks = 0;
  st->flagged_argmins = 0;
}

// ------------------------------------------------------------------ gather
template <typename T>
__global__ __launch_bounds__(256) void kb_gather(const kmpar_instance* inst, int rounds, PlanPtrs p,
                                                 int t) {
  const BView v = bview(inst, blockIdx.x, p, rounds);
  const int d = v.I->d, DP = padded_dim_hd(d);
  const int* rs = v.at<int>(v.r.rs);
  const int id0 = rs[t], m = rs[t + 1] - id0;
  const int* cand = v.at<int>(v.r.cand);
  float* Call = v.at<float>(v.r.Call);
  float* CallT = v.at<float>(v.r.CallT);
  const int64_t ldT = v.r.capT;
  const T* X = static_cast<const T*>(v.I->X);
  for (int idx = threadIdx.x; idx < m * DP; idx += 256) {
    const int j = idx / DP, e = idx - j * DP;
    const int pt = cand[id0 + j];
    const float x =
        e < d ? Elem<T>::get(X, (int64_t)pt * d + e, row_scale_of<T>(v.I->row_scale, pt)) : 0.0f;
    Call[(int64_t)(id0 + j) * DP + e] = x;
    CallT[(int64_t)e * ldT + id0 + j] = x;
  }
}

// ---------------------------------------------------------------- the fold
// Same per-point arithmetic as k_fold_direct: candidates in id order, strict
// improvement, FP32 direct form.
template <int DP, typename T, int CB>
__global__ __launch_bounds__(kBFold) void kb_fold(const kmpar_instance* inst, int rounds,
                                                  PlanPtrs p, int g, int t, int first) {
  constexpr int DCH = DP <= 128 ? DP : DP / 2;
  constexpr int NCH = DP / DCH;
  const int gb = p.gbeg[g], gn = p.gbeg[g + 1] - gb;
  const int* pre = p.gpre + gb + g;
  const int q = find_owner(pre, gn, blockIdx.x);
  const int ii = p.glist[gb + q];
  const BView v = bview(inst, ii, p, rounds);
  const int i = (blockIdx.x - pre[q]) * kBFold + threadIdx.x;
  const int n = (int)v.I->n, d = v.I->d;
  if (i >= n) return;
  const int* rs = v.at<int>(v.r.rs) + t;
  const int id0 = rs[0], m = rs[1] - id0;
  const float* __restrict__ C = v.at<const float>(v.r.Call) + (int64_t)id0 * DP;
  const T* __restrict__ X = static_cast<const T*>(v.I->X);
  const float sc = row_scale_of<T>(v.I->row_scale, i);
  const int64_t row = (int64_t)i * d;
  float best = INFINITY;
  int bj = -1;
  // CB candidates per step, each an independent chain of FMAs (the tile
  // shape the batch's tuner chooses); candidates in id order, the first
  // strictly smallest kept, so every CB gives the same result.
  if constexpr (NCH == 1) {
    float x[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) x[j] = (j < d) ? Elem<T>::get(X, row + j, sc) : 0.0f;
    for (int c0 = 0; c0 < m; c0 += CB) {
      float acc[CB];
#pragma unroll
      for (int qq = 0; qq < CB; ++qq) {
        acc[qq] = 0.0f;
        if (c0 + qq < m) {
          const float* __restrict__ cr = C + (int64_t)(c0 + qq) * DP;
#pragma unroll
          for (int j = 0; j < DP; ++j) {
            const float tt = x[j] - cr[j];
            acc[qq] = fmaf(tt, tt, acc[qq]);
          }
        }
      }
#pragma unroll
      for (int qq = 0; qq < CB; ++qq)
        if (c0 + qq < m && acc[qq] < best) {
          best = acc[qq];
          bj = c0 + qq;
        }
    }
  } else {
    for (int c0 = 0; c0 < m; c0 += CB) {
      float acc[CB];
#pragma unroll
      for (int qq = 0; qq < CB; ++qq) acc[qq] = 0.0f;
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        float x[DCH];
#pragma unroll
        for (int j = 0; j < DCH; ++j) {
          const int jj = h * DCH + j;
          x[j] = (jj < d) ? Elem<T>::get(X, row + jj, sc) : 0.0f;
        }
#pragma unroll
        for (int qq = 0; qq < CB; ++qq) {
          if (c0 + qq < m) {
            const float* __restrict__ cr = C + (int64_t)(c0 + qq) * DP + h * DCH;
#pragma unroll
            for (int j = 0; j < DCH; ++j) {
              const float tt = x[j] - cr[j];
              acc[qq] = fmaf(tt, tt, acc[qq]);
            }
          }
        }
      }
#pragma unroll
      for (int qq = 0; qq < CB; ++qq)
        if (c0 + qq < m && acc[qq] < best) {
          best = acc[qq];
          bj = c0 + qq;
        }
    }
  }
  float* D2 = v.at<float>(v.r.D2);
  int* A = v.at<int>(v.r.A);
  if (first) {
    D2[i] = best;
    A[i] = bj >= 0 ? id0 + bj : -1;
  } else if (bj >= 0 && best < D2[i]) {
    D2[i] = best;
    A[i] = id0 + bj;
  }
}

// The same fold for rows of 65 to 128 padded elements, each row split over
// two waves: a block of 2 * kBFold threads holds its 256 points in four pairs
// of waves, the first wave of a pair with elements [0, 64) of its 64 points'
// rows in registers, the second with [64, DP). Per chunk of kPairChunk
// candidates the first wave runs the FMA chain over its elements and leaves
// each partial sum in LDS; one chunk later the second wave continues the same
// chain from it over the rest of the row and keeps the best candidate. The
// chain is kb_fold's, in the same order, so the result is bitwise the same;
// each wave needs half the row registers and reads 64 row elements per
// candidate, as the fold of 64-element rows does.
constexpr int kPairChunk = 16;

template <int DP, typename T>
__global__ __launch_bounds__(2 * kBFold) void kb_fold_pair(const kmpar_instance* inst, int rounds,
                                                           PlanPtrs p, int g, int t, int first) {
  static_assert(DP > 64 && DP <= 128, "rows of 65 to 128 padded elements");
  constexpr int H1 = DP - 64, CH = kPairChunk;
  __shared__ float part[2][CH][kBFold];  // [buffer][candidate of the chunk][point of the block]
  const int gb = p.gbeg[g], gn = p.gbeg[g + 1] - gb;
  const int* pre = p.gpre + gb + g;
  const int q = find_owner(pre, gn, blockIdx.x);
  const int ii = p.glist[gb + q];
  const BView v = bview(inst, ii, p, rounds);
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int half = wv / 4;                    // 0: elements [0, 64); 1: [64, DP)
  const int pl = (wv % 4) * kWave + lane;     // the point within the block
  const int i = (blockIdx.x - pre[q]) * kBFold + pl;
  const int n = (int)v.I->n, d = v.I->d;
  const bool live = i < n;                    // every wave takes part in the barriers
  const int* rs = v.at<int>(v.r.rs) + t;
  const int id0 = rs[0], m = rs[1] - id0;
  const float* __restrict__ C = v.at<const float>(v.r.Call) + (int64_t)id0 * DP;
  const T* __restrict__ X = static_cast<const T*>(v.I->X);
  const float sc = live ? row_scale_of<T>(v.I->row_scale, i) : 1.0f;
  const int64_t row = (int64_t)i * d;
  const int e0 = half ? 64 : 0;
  float x[64];
#pragma unroll
  for (int j = 0; j < 64; ++j)
    x[j] = (live && e0 + j < d) ? Elem<T>::get(X, row + e0 + j, sc) : 0.0f;
  float best = INFINITY;
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
            const float tt = x[e] - cr[e];
            acc = fmaf(tt, tt, acc);
          }
          dst[jj * kBFold] = acc;
        }
      }
    } else if (it > 0) {
      const int c0 = (it - 1) * CH, nc = min(CH, m - c0);
      const float* src = &part[(it - 1) & 1][0][pl];
      for (int jj = 0; jj < nc; ++jj) {
        const float* __restrict__ cr = C + (int64_t)(c0 + jj) * DP + 64;
        float acc = src[jj * kBFold];
#pragma unroll
        for (int e = 0; e < H1; ++e) {
          const float tt = x[e] - cr[e];
          acc = fmaf(tt, tt, acc);
        }
        if (acc < best) {
          best = acc;
          bj = c0 + jj;
        }
      }
    }
    __syncthreads();  // chunk it written, chunk it - 1 consumed
  }
  if (half == 0 || !live) return;
  float* D2 = v.at<float>(v.r.D2);
  int* A = v.at<int>(v.r.A);
  if (first) {
    D2[i] = best;
    A[i] = bj >= 0 ? id0 + bj : -1;
  } else if (bj >= 0 && best < D2[i]) {
    D2[i] = best;
    A[i] = id0 + bj;
  }
}

// -------------------------------------------------------------------- phi
__global__ __launch_bounds__(256) void kb_phi_partial(const kmpar_instance* inst, int count,
                                                      int rounds, PlanPtrs p) {
  __shared__ double sh[8];
  const int ii = find_owner(p.pre_phi, count, blockIdx.x);
  const BView v = bview(inst, ii, p, rounds);
  const int chunk = blockIdx.x - p.pre_phi[ii];
  const int n = (int)v.I->n;
  const float* D2 = v.at<float>(v.r.D2);
  double acc = 0.0;
  for (int r = 0; r < kPhiChunk / 256; ++r) {
    const int i = chunk * kPhiChunk + r * 256 + threadIdx.x;
    if (i < n) acc += (double)D2[i];
  }
  const double tot = block_sum<double, 256>(acc, sh);
  if (threadIdx.x == 0) v.at<double>(v.r.phi_part)[chunk] = tot;
}

__global__ __launch_bounds__(256) void kb_phi_final(const kmpar_instance* inst, int rounds,
                                                    PlanPtrs p, int t) {
  __shared__ double sh[8];
  const BView v = bview(inst, blockIdx.x, p, rounds);
  const int nb = (int)((v.I->n + kPhiChunk - 1) / kPhiChunk);
  const double* part = v.at<double>(v.r.phi_part);
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  const double tot = block_sum<double, 256>(acc, sh);
  if (threadIdx.x == 0) v.at<kmpar_stats>(v.r.st)->phi[t] = tot;
}

// -------------------------------------------------------------------- draw
// Round t's draw of point i (Algorithm 2 step 4); *flag as in the
// single-instance draw: |u - p| <= band * p.
__device__ __forceinline__ int bkeep(const float* D2, int i, double phi, double ell, uint64_t seed,
                                     int t, uint64_t inst, double band = 0.0,
                                     int* flag = nullptr) {
  if (flag) *flag = 0;
  if (!(phi > 0.0)) return 0;
  double pr = ell * (double)D2[i] / phi;
  if (pr > 1.0) pr = 1.0;
  const double u = philox_uniform(seed, kTagRound, (uint64_t)i, (uint64_t)t, inst);
  if (flag) *flag = (pr > 0.0 && fabs(u - pr) <= band * pr) ? 1 : 0;
  return u < pr ? 1 : 0;
}

__global__ __launch_bounds__(256) void kb_draw_count(const kmpar_instance* inst, int count,
                                                     int rounds, PlanPtrs p, uint64_t seed, int t) {
  __shared__ int sh[8];
  const int ii = find_owner(p.pre_draw, count, blockIdx.x);
  const BView v = bview(inst, ii, p, rounds);
  const int chunk = blockIdx.x - p.pre_draw[ii];
  const int n = (int)v.I->n;
  const float* D2 = v.at<float>(v.r.D2);
  kmpar_stats* st = v.at<kmpar_stats>(v.r.st);
  const double phi = st->phi[t - 1];
  const double band = fp32_flag_band(v.I->d);
  int c = 0, nf = 0;
  for (int r = 0; r < kDrawChunk / 256; ++r) {
    const int i = chunk * kDrawChunk + r * 256 + threadIdx.x;
    if (i < n) {
      int fl = 0;
      c += bkeep(D2, i, phi, v.I->ell, seed, t, (uint64_t)ii, band, &fl);
      nf += fl;
    }
  }
  const int tot = block_sum<int, 256>(c, sh);
  if (threadIdx.x == 0) v.at<int>(v.r.cnt)[chunk] = tot;
  const int ftot = block_sum<int, 256>(nf, sh);
  if (threadIdx.x == 0 && ftot) atomicAdd(&st->flagged_draws, ftot);
}

// Per instance: exclusive scan of its chunk counts and commit of round t.
__global__ __launch_bounds__(1024) void kb_scan_commit(const kmpar_instance* inst, int rounds,
                                                       PlanPtrs p, int t) {
  __shared__ long long sh[17];
  const BView v = bview(inst, blockIdx.x, p, rounds);
  const int L = (int)((v.I->n + kDrawChunk - 1) / kDrawChunk);
  int* a = v.at<int>(v.r.cnt);
  const int R = (L + 1023) / 1024;
  const int lo = min(L, (int)threadIdx.x * R), hi = min(L, lo + R);
  long long s = 0;
  for (int j = lo; j < hi; ++j) s += a[j];
  long long tot;
  long long run = block_excl_scan<long long, 1024>(s, sh, &tot);
  for (int j = lo; j < hi; ++j) {
    const int x = a[j];
    a[j] = (int)run;
    run += x;
  }
  if (threadIdx.x == 0) {
    const int cap = (int)cap_round_hd(v.I->n, v.I->ell);
    int* rs = v.at<int>(v.r.rs);
    kmpar_stats* st = v.at<kmpar_stats>(v.r.st);
    const int m = tot < cap ? (int)tot : cap;
    rs[t + 1] = rs[t] + m;
    st->round_count[t] = m;
    if (tot > cap) st->status = KMPAR_E_OVERFLOW;
  }
}

__global__ __launch_bounds__(256) void kb_draw_write(const kmpar_instance* inst, int count,
                                                     int rounds, PlanPtrs p, uint64_t seed, int t) {
  __shared__ int sh[8];
  const int ii = find_owner(p.pre_draw, count, blockIdx.x);
  const BView v = bview(inst, ii, p, rounds);
  const int chunk = blockIdx.x - p.pre_draw[ii];
  const int n = (int)v.I->n;
  const float* D2 = v.at<float>(v.r.D2);
  const double phi = v.at<kmpar_stats>(v.r.st)->phi[t - 1];
  const int cap = (int)cap_round_hd(v.I->n, v.I->ell);
  int run = v.at<int>(v.r.cnt)[chunk];
  const int start = v.at<int>(v.r.rs)[t];
  int* cand = v.at<int>(v.r.cand);
  for (int r = 0; r < kDrawChunk / 256; ++r) {
    const int i = chunk * kDrawChunk + r * 256 + threadIdx.x;
    const int keep = (i < n) ? bkeep(D2, i, phi, v.I->ell, seed, t, (uint64_t)ii) : 0;
    int tot;
    const int rank = block_excl_scan<int, 256>(keep, sh, &tot);
    if (keep && run + rank < cap) cand[start + run + rank] = i;
    run += tot;
  }
}

// ----------------------------------------------------------------- weights
__global__ __launch_bounds__(256) void kb_zero_w(const kmpar_instance* inst, int rounds, PlanPtrs p) {
  const BView v = bview(inst, blockIdx.x, p, rounds);
  const int nc = v.at<int>(v.r.rs)[rounds + 1];
  kmpar_stats* st = v.at<kmpar_stats>(v.r.st);
  if (threadIdx.x == 0) st->n_candidates = nc;
  int* w = v.at<int>(v.r.w);
  for (int j = threadIdx.x; j < nc; j += 256) w[j] = 0;
}

__global__ __launch_bounds__(256) void kb_hist(const kmpar_instance* inst, int count, int rounds,
                                               PlanPtrs p) {
  const int ii = find_owner(p.pre_draw, count, blockIdx.x);
  const BView v = bview(inst, ii, p, rounds);
  const int chunk = blockIdx.x - p.pre_draw[ii];
  const int n = (int)v.I->n;
  const int nc = v.at<int>(v.r.rs)[rounds + 1];
  const int* A = v.at<int>(v.r.A);
  int* w = v.at<int>(v.r.w);
  for (int r = 0; r < kDrawChunk / 256; ++r) {
    const int i = chunk * kDrawChunk + r * 256 + threadIdx.x;
    if (i < n) {
      const int a = A[i];
      if (a >= 0 && a < nc) atomicAdd(&w[a], 1);
    }
  }
}

// --------------------------------------------------------------- recluster
__global__ __launch_bounds__(kBRecl) void kb_recluster(const kmpar_instance* inst, int rounds,
                                                       PlanPtrs p, uint64_t seed, int cap_lds) {
  extern __shared__ float lds[];
  const int ii = blockIdx.x;
  const BView v = bview(inst, ii, p, rounds);
  const int d = v.I->d;
  recluster_block<kBRecl>(v.at<const float>(v.r.CallT), (int)v.r.capT, d, v.at<const int>(v.r.w),
                          v.at<int>(v.r.rs)[rounds + 1], v.I->k, seed, (uint64_t)ii,
                          v.at<int>(v.r.picks), v.I->centers, v.at<kmpar_stats>(v.r.st), lds,
                          cap_lds, fp32_flag_band(d));
}

// Optional per-instance trace copies (one workgroup per instance).
__global__ __launch_bounds__(256) void kb_trace(const kmpar_instance* inst, int rounds, PlanPtrs p,
                                                const kmpar_trace* tr) {
  const BView v = bview(inst, blockIdx.x, p, rounds);
  const kmpar_trace t = tr[blockIdx.x];
  const kmpar_stats* st = v.at<kmpar_stats>(v.r.st);
  const int nc = st->n_candidates, nk = st->n_centers, n = (int)v.I->n;
  for (int j = threadIdx.x; j < nc; j += 256) {
    if (t.cand_point) t.cand_point[j] = v.at<int>(v.r.cand)[j];
    if (t.cand_weight) t.cand_weight[j] = v.at<int>(v.r.w)[j];
  }
  for (int j = threadIdx.x; j < nk; j += 256)
    if (t.center_cand) t.center_cand[j] = v.at<int>(v.r.picks)[j];
  for (int j = threadIdx.x; j < n; j += 256) {
    if (t.assign) t.assign[j] = v.at<int>(v.r.A)[j];
    if (t.d2) t.d2[j] = v.at<float>(v.r.D2)[j];
  }
}

__global__ void kb_copy_stats(const kmpar_instance* inst, int count, int rounds, PlanPtrs p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const BView v = bview(inst, i, p, rounds);
  if (v.I->stats) *v.I->stats = *v.at<kmpar_stats>(v.r.st);
}

// ------------------------------------------------------------------ host
size_t batched_recluster_lds(const kmpar_instance* ih, int count, int rounds);

size_t batched_workspace(const kmpar_instance* inst, int count, int rounds, int* G_out,
                         int* dps) {
  int G = 0;
  int64_t total = 0;
  for (int i = 0; i < count; ++i) {
    total += region_of(inst[i].n, inst[i].d, inst[i].k, inst[i].ell, rounds).bytes;
    const int dp = padded_dim_hd(inst[i].d);
    bool seen = false;
    for (int g = 0; g < G; ++g) seen |= dps[g] == dp;
    if (!seen) dps[G++] = dp;
  }
  // groups in increasing padded dim
  for (int a = 0; a < G; ++a)
    for (int b = a + 1; b < G; ++b)
      if (dps[b] < dps[a]) {
        const int t = dps[a];
        dps[a] = dps[b];
        dps[b] = t;
      }
  *G_out = G;
  const PlanPtrs pp = plan_ptrs(nullptr, count, G);
  return (size_t)(pp.regions - (char*)nullptr) + (size_t)total;
}

// Fold variants the tuner tries: rows of up to 128 padded elements held
// whole in registers (1, 2 or 4 candidates per step), rows of 65 to 128 also
// split over two waves (kCbPair, the default there: 292 -> 230 ms for the
// 1,024-instance batch), wider rows in two halves (4 or 8).
constexpr int kCbNarrow[3] = {1, 2, 4};
constexpr int kCbWide[2] = {4, 8};
constexpr int kCbPair = 200;  // kb_fold_pair, rows of 65 to 128 padded elements
constexpr int kCbMaxVariants = 4;
static int batch_cb_default(int DP) { return DP <= 64 ? 1 : DP <= 128 ? kCbPair : 8; }
static int batch_cb_variants(int DP, int* out) {
  if (DP <= 128) {
    for (int i = 0; i < 3; ++i) out[i] = kCbNarrow[i];
    if (DP > 64) {
      out[3] = kCbPair;
      return 4;
    }
    return 3;
  }
  for (int i = 0; i < 2; ++i) out[i] = kCbWide[i];
  return 2;
}

template <int DP, typename T, int CB>
static void launch_bfold(const kmpar_instance* inst, int rounds, const PlanPtrs& p, int g, int t,
                         int first, int tiles, hipStream_t s) {
  hipLaunchKernelGGL((kb_fold<DP, T, CB>), dim3(tiles), dim3(kBFold), 0, s, inst, rounds, p, g, t,
                     first);
}

template <int DP, typename T>
static hipError_t launch_bfold_cb(int cb, const kmpar_instance* inst, int rounds, const PlanPtrs& p,
                                  int g, int t, int first, int tiles, hipStream_t s) {
  if constexpr (DP <= 128) {
    switch (cb) {
      case 1: launch_bfold<DP, T, 1>(inst, rounds, p, g, t, first, tiles, s); return hipSuccess;
      case 2: launch_bfold<DP, T, 2>(inst, rounds, p, g, t, first, tiles, s); return hipSuccess;
      case 4: launch_bfold<DP, T, 4>(inst, rounds, p, g, t, first, tiles, s); return hipSuccess;
    }
    if constexpr (DP > 64) {
      if (cb == kCbPair) {
        hipLaunchKernelGGL((kb_fold_pair<DP, T>), dim3(tiles), dim3(2 * kBFold), 0, s, inst, rounds,
                           p, g, t, first);
        return hipSuccess;
      }
    }
  } else {
    switch (cb) {
      case 4: launch_bfold<DP, T, 4>(inst, rounds, p, g, t, first, tiles, s); return hipSuccess;
      case 8: launch_bfold<DP, T, 8>(inst, rounds, p, g, t, first, tiles, s); return hipSuccess;
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_bfold_dp(int DP, int cb, const kmpar_instance* inst, int rounds,
                                  const PlanPtrs& p, int g, int t, int first, int tiles,
                                  hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  hipError_t e = hipErrorInvalidValue;
  switch (DP) {
#define KMPAR_CASE(V) \
  case V: e = launch_bfold_cb<V, T>(cb, inst, rounds, p, g, t, first, tiles, s); break;
    KMPAR_CASE(4) KMPAR_CASE(8) KMPAR_CASE(12) KMPAR_CASE(16) KMPAR_CASE(20) KMPAR_CASE(24)
    KMPAR_CASE(28) KMPAR_CASE(32) KMPAR_CASE(36) KMPAR_CASE(40) KMPAR_CASE(44) KMPAR_CASE(48)
    KMPAR_CASE(52) KMPAR_CASE(56) KMPAR_CASE(60) KMPAR_CASE(64) KMPAR_CASE(80) KMPAR_CASE(96)
    KMPAR_CASE(112) KMPAR_CASE(128) KMPAR_CASE(160) KMPAR_CASE(192) KMPAR_CASE(224)
    KMPAR_CASE(256)
#undef KMPAR_CASE
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// Times every candidate-block variant of group g's fold of round t (the
// launches re-apply the same fold, which changes nothing after the first)
// and returns the fastest; the stream is synchronised once.
template <typename T>
static hipError_t tune_bfold(int DP, const kmpar_instance* inst, int rounds, const PlanPtrs& p,
                             int g, int t, int tiles, hipStream_t s, int* best_cb) {
  int vars[kCbMaxVariants];
  const int nv = batch_cb_variants(DP, vars);
  hipEvent_t ev[kCbMaxVariants + 1];
  for (int i = 0; i <= nv; ++i) {
    hipError_t e = hipEventCreate(&ev[i]);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      return e;
    }
  }
  hipError_t e = hipEventRecord(ev[0], s);
  for (int i = 0; i < nv && e == hipSuccess; ++i) {
    e = launch_bfold_dp<T>(DP, vars[i], inst, rounds, p, g, t, 0, tiles, s);
    if (e == hipSuccess) e = hipEventRecord(ev[i + 1], s);
  }
  if (e == hipSuccess) e = hipEventSynchronize(ev[nv]);
  float best_ms = 0.0f;
  *best_cb = vars[0];
  for (int i = 0; i < nv && e == hipSuccess; ++i) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
    if (e == hipSuccess && (i == 0 || ms < best_ms)) {
      best_ms = ms;
      *best_cb = vars[i];
    }
  }
  for (int i = 0; i <= nv; ++i) (void)hipEventDestroy(ev[i]);
  return e;
}

template <typename T>
static hipError_t run_batched_t(kmpar_dtype dt, const kmpar_instance* ih, const kmpar_instance* idev,
                                int count, int rounds, uint64_t seed, void* ws,
                                const kmpar_trace* tr, BatchTuner* tuner,
                                const LaunchTimer* fold_timer, hipStream_t s) {
  auto fold = [&](const std::function<hipError_t()>& launch) {
    return fold_timer ? (*fold_timer)(launch) : launch();
  };
  int dps[kBatchMaxGroups];
  int G = 0;
  (void)batched_workspace(ih, count, rounds, &G, dps);
  GroupTable gt{};
  gt.G = G;
  for (int g = 0; g < G; ++g) gt.dp[g] = dps[g];
  const PlanPtrs p = plan_ptrs(ws, count, G);
  // host copies of the work-list sizes (the device builds the same lists)
  long long draw_blocks = 0, phi_blocks = 0;
  int gtiles[kBatchMaxGroups] = {0};
  int64_t max_cap = 0, max_k = 0;
  for (int i = 0; i < count; ++i) {
    draw_blocks += (ih[i].n + kDrawChunk - 1) / kDrawChunk;
    phi_blocks += (ih[i].n + kPhiChunk - 1) / kPhiChunk;
    const int dp = padded_dim_hd(ih[i].d);
    for (int g = 0; g < G; ++g)
      if (dps[g] == dp) gtiles[g] += (int)((ih[i].n + kBFold - 1) / kBFold);
    const int64_t capT = 1 + (int64_t)rounds * cap_round_hd(ih[i].n, ih[i].ell);
    if (capT > max_cap) max_cap = capT;
    if (ih[i].k > max_k) max_k = ih[i].k;
  }
  // tile shapes: the tuner's choice per (dtype, padded row length), tuned on
  // round 1 the first time a shape is seen (never under stream capture)
  int gcb[kBatchMaxGroups];
  bool gtune[kBatchMaxGroups];
  bool can_tune = tuner && tuner->enabled;
  if (can_tune) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      can_tune = false;
  }
  for (int g = 0; g < G; ++g) {
    const int key = BatchTuner::key((int)dt, dps[g]);
    const bool known = tuner && tuner->cb.count(key) != 0;
    gcb[g] = known ? tuner->cb.at(key) : batch_cb_default(dps[g]);
    gtune[g] = can_tune && !known && rounds >= 1;
  }
  const dim3 per_inst(count), inst_threads((count + 255) / 256);
  hipLaunchKernelGGL(kb_plan, dim3(1), dim3(1024), 0, s, idev, count, rounds, gt, p);
  hipLaunchKernelGGL(kb_first, inst_threads, dim3(256), 0, s, idev, count, rounds, p, seed);
  hipLaunchKernelGGL(kb_gather<T>, per_inst, dim3(256), 0, s, idev, rounds, p, 0);
  for (int g = 0; g < G; ++g) {
    hipError_t e = fold([&] {
      return launch_bfold_dp<T>(dps[g], gcb[g], idev, rounds, p, g, 0, 1, gtiles[g], s);
    });
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kb_phi_partial, dim3((unsigned)phi_blocks), dim3(256), 0, s, idev, count,
                     rounds, p);
  hipLaunchKernelGGL(kb_phi_final, per_inst, dim3(256), 0, s, idev, rounds, p, 0);
  for (int t = 1; t <= rounds; ++t) {
    hipLaunchKernelGGL(kb_draw_count, dim3((unsigned)draw_blocks), dim3(256), 0, s, idev, count,
                       rounds, p, seed, t);
    hipLaunchKernelGGL(kb_scan_commit, per_inst, dim3(1024), 0, s, idev, rounds, p, t);
    hipLaunchKernelGGL(kb_draw_write, dim3((unsigned)draw_blocks), dim3(256), 0, s, idev, count,
                       rounds, p, seed, t);
    hipLaunchKernelGGL(kb_gather<T>, per_inst, dim3(256), 0, s, idev, rounds, p, t);
    for (int g = 0; g < G; ++g) {
      hipError_t e;
      if (t == 1 && gtune[g] && gtiles[g] > 0) {
        e = tune_bfold<T>(dps[g], idev, rounds, p, g, t, gtiles[g], s, &gcb[g]);
        if (e == hipSuccess) tuner->cb[BatchTuner::key((int)dt, dps[g])] = gcb[g];
      } else {
        e = fold([&] {
          return launch_bfold_dp<T>(dps[g], gcb[g], idev, rounds, p, g, t, 0, gtiles[g], s);
        });
      }
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kb_phi_partial, dim3((unsigned)phi_blocks), dim3(256), 0, s, idev, count,
                       rounds, p);
    hipLaunchKernelGGL(kb_phi_final, per_inst, dim3(256), 0, s, idev, rounds, p, t);
  }
  hipLaunchKernelGGL(kb_zero_w, per_inst, dim3(256), 0, s, idev, rounds, p);
  hipLaunchKernelGGL(kb_hist, dim3((unsigned)draw_blocks), dim3(256), 0, s, idev, count, rounds, p);
  const size_t lds = batched_recluster_lds(ih, count, rounds);
  hipError_t e = hipFuncSetAttribute((const void*)kb_recluster,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_recluster, per_inst, dim3(kBRecl), lds, s, idev, rounds, p, seed,
                     (int)max_cap);
  if (tr) hipLaunchKernelGGL(kb_trace, per_inst, dim3(256), 0, s, idev, rounds, p, tr);
  hipLaunchKernelGGL(kb_copy_stats, inst_threads, dim3(256), 0, s, idev, count, rounds, p);
  return hipGetLastError();
}

hipError_t launch_batched(kmpar_dtype dt, const kmpar_instance* ih, const kmpar_instance* idev,
                          int count, int rounds, uint64_t seed, void* ws, const kmpar_trace* tr,
                          BatchTuner* tuner, const LaunchTimer* fold_timer, hipStream_t s) {
  switch (dt) {
    case KMPAR_F32:
      return run_batched_t<float>(dt, ih, idev, count, rounds, seed, ws, tr, tuner, fold_timer, s);
    case KMPAR_BF16:
      return run_batched_t<bf16_t>(dt, ih, idev, count, rounds, seed, ws, tr, tuner, fold_timer, s);
    case KMPAR_FP8_E4M3:
      return run_batched_t<fp8_t>(dt, ih, idev, count, rounds, seed, ws, tr, tuner, fold_timer, s);
  }
  return hipErrorInvalidValue;
}

size_t batched_recluster_lds(const kmpar_instance* ih, int count, int rounds) {
  int64_t max_cap = 0, max_k = 0;
  for (int i = 0; i < count; ++i) {
    const int64_t capT = 1 + (int64_t)rounds * cap_round_hd(ih[i].n, ih[i].ell);
    if (capT > max_cap) max_cap = capT;
    if (ih[i].k > max_k) max_k = ih[i].k;
  }
  return (size_t)max_cap * 8 + (size_t)max_k * 8;
}

}  // namespace kmpar
