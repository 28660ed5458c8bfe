// REFINED distance pass: an MFMA screen with a rigorous lower bound, then an
// FP32 direct-form refinement of the screen winner; points the bound cannot
// settle are listed and recomputed by the direct-form fold.
//
// For point x and candidate c, t = ||x - c||^2 = ||x||^2 + ||c||^2 - 2 x.c.
// The screen forms x.c on the matrix cores from bf16 operands (exact bf16
// inputs, or a two/three-term bf16 split of FP32 values, products exact and
// summed in FP32) and the lower bound
//   lb = (1 - 2G)(||x||^2 + ||c||^2) - 2 x.c   <=  t  - (direct-form error),
// where 2G (||x||^2 + ||c||^2) bounds every rounding error of the screen and of
// the FP32 direct form (host code derives G from d, K and the split).  Per
// point the kernel keeps the smallest and second smallest lb and the argmin
// j1, refines t(j1) = r1 exactly as the plain kernel would, and then:
//   lb_min >= D2                      -> no candidate can be strictly closer;
//   r1 <  D2 and lb_2nd >  r1         -> j1 is the unique nearest: fold it in;
//   r1 >= D2 and lb_2nd >= D2         -> no candidate is strictly closer;
//   otherwise                         -> the point is listed for a full
//                                        direct-form pass over the candidates.
// Every decision is therefore the decision of the FP32 direct-form path.
//
// Within a group of up to 64 candidate tiles (one or more LDS chunks), the
// running maxima carry the tile's position in the group in the low TB
// mantissa bits of the value itself (the lane fixes the column within the
// tile), so the per-value work is one bit insert and two med3; each group's
// maxima are then merged with explicit ids.  Replacing those bits moves acc by less than 2^(TB-23) |acc| <=
// 2^(TB-23) S, S = ||x||^2 + ||c||^2, which the budget of G includes.  The bound also
// assumes no overflow and negligible underflow: points with ||x||^2 outside
// [2^-100, 2^100] are always listed, and candidates with ||c||^2 > 2^100
// get a trivial bound (every point refines or lists them).
//
// FP8 rows (e4m3 codes q with a row scale s, element = fl(s * q)) enter the
// matrix cores as their codes, which bf16 holds exactly, against the codes
// of candidate rows of X: the products q_x . q_c are exact.  The
// accumulators start at zero and each value is then scaled,
// acc * (s_x * s_c) - ncg_c / 2, which the budget of G covers with the
// roundings of the scales.  Rows whose scale lies outside [2^-63, 2^63] are
// listed; candidates whose scale does get a trivial bound.  (Assignment
// passes of FP8 rows against FP32 centers use the direct form.)
#include <float.h>
#include <cmath>
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"
#include "rows.hpp"

namespace kmpar {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Range of squared norms inside which the screen's error budget holds.
constexpr float kNormMax = 0x1p100f;
constexpr float kNormMin = 0x1p-100f;

// FP32 -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Range of row scales inside which the scaled epilogue cannot overflow.
constexpr float kScaleMin = 0x1p-63f;
constexpr float kScaleMax = 0x1p63f;

// bf16 bits of an e4m3 code's value (exact: four significant bits).
__device__ __forceinline__ uint16_t code_bf16(uint8_t q) {
  return (uint16_t)(__float_as_uint(decode_e4m3(q)) >> 16);
}

// Element idx as the A operand takes it: the decoded element, or the
// unscaled code of an FP8 row.
template <typename T>
__device__ __forceinline__ float op_elem(const T* X, int64_t idx, float decoded) {
  return decoded;
}
template <>
__device__ __forceinline__ float op_elem<fp8_t>(const fp8_t* X, int64_t idx, float) {
  return decode_e4m3(X[idx].bits);
}

// Operand k of the screen's K axis.  SPLIT 1: A = x, B = c (both exact in
// bf16).  SPLIT 2: A = [x | x], B = [hi(c) | lo(c)].  SPLIT 3: A = [hi(x) |
// lo(x) | hi(x)], B = [hi(c) | hi(c) | lo(c)].  k >= SPLIT*d is zero.
template <int SPLIT>
__device__ __forceinline__ uint16_t a_elem(float x, int part) {
  if constexpr (SPLIT == 3) {
    const uint16_t h = bf16_rne(x);
    return part == 1 ? bf16_rne(x - bf16_val(h)) : h;
  } else {
    return bf16_rne(x);
  }
}
template <int SPLIT>
__device__ __forceinline__ uint16_t b_elem(float c, int part) {
  const uint16_t h = bf16_rne(c);
  if constexpr (SPLIT == 1) return h;
  const uint16_t l = bf16_rne(c - bf16_val(h));
  if constexpr (SPLIT == 2) return part == 0 ? h : l;
  return part == 2 ? l : h;
}

// --------------------------------------------------------------- B operands
// One wave per tile of 16 candidates: writes KS k-steps of 64 lanes x 8 bf16
// in the lane order the MFMA B operand uses (lane l: candidate l%16,
// k = s*32 + (l/16)*8 + e), plus ncg_j = (1 - 2G) ||c_j||^2 (+inf past m).
// CODES: the operands are the e4m3 codes of X row cand[id0 + j] (SPLIT 1),
// and scg receives each candidate's row scale, 0 past m or when the scale
// is outside the screen's range (then the bias is trivial as well).
// Block 0 also hands the previous pass's listed count to the stats and
// clears it for the screen that follows.
template <int SPLIT, int KS, bool CODES>
__global__ __launch_bounds__(64) void k_prep_b(const float* C, int DP, int d, const int* rs,
                                               int m_host, float oneminus2g, u16x8* B,
                                               float* ncg, const fp8_t* Xc, const float* rsc,
                                               const int* cand, float* scg, int* list_len,
                                               kmpar_stats* st, const int* cperm) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && list_len) {
    if (st) st->n_rescanned += *list_len;
    *list_len = 0;
  }
  int id0 = 0, m = m_host;
  if (rs) {
    id0 = rs[0];
    m = rs[1] - id0;
  }
  const int q = blockIdx.x;
  if (q * 16 >= m) return;
  const int lane = threadIdx.x;
  const int j = q * 16 + (lane % 16);  // position in the pass's tiles
  const bool valid = j < m;
  const int src = valid ? (cperm ? cperm[j] : j) : 0;  // the candidate at position j
  const float* c = C + (int64_t)(id0 + src) * DP;
  int64_t xrow = 0;
  if constexpr (CODES) xrow = valid ? (int64_t)cand[id0 + src] * d : 0;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    u16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = s * 32 + (lane / 16) * 8 + e;
      const int part = k / d, coord = k - part * d;
      if constexpr (CODES)
        v[e] = (valid && part < SPLIT) ? code_bf16(Xc[xrow + coord].bits) : (uint16_t)0;
      else
        v[e] = (valid && part < SPLIT) ? b_elem<SPLIT>(c[coord], part) : (uint16_t)0;
    }
    B[((int64_t)q * KS + s) * 64 + lane] = v;
  }
  if (lane < 16) {
    float nc = 0.0f;
    if (valid)
      for (int e = 0; e < d; ++e) nc = fmaf(c[e], c[e], nc);
    float sc = 1.0f;
    if constexpr (CODES) sc = valid ? rsc[cand[id0 + src]] : 0.0f;
    const bool sc_ok = sc >= kScaleMin && sc <= kScaleMax;
    // Past m: +inf (never the maximum).  Beyond 2^100 (or not finite), or a
    // scale out of range: a bias that makes the candidate's lower bound -inf.
    ncg[j] = !valid ? INFINITY : (nc <= kNormMax && sc_ok ? oneminus2g * nc : -FLT_MAX);
    if constexpr (CODES) scg[j] = (valid && sc_ok) ? sc : 0.0f;
  }
}

// ||x||^2 of a staged row: FP32 fmas over the coordinates in ascending order.
__device__ __forceinline__ float staged_norm(const float* xr, int d) {
  float nx = 0.0f;
#pragma unroll 8
  for (int e = 0; e < d; ++e) nx = fmaf(xr[e], xr[e], nx);
  return nx;
}

// --------------------------------------------------------------- A operands
// The A operands of a block's 64 staged rows: for every tile of 16 points and
// k-step s, 64 lanes x 8 bf16 in the lane order of the MFMA A operand (lane
// l: point l%16, k = s*32 + (l/16)*8 + e, split term k / d of coordinate
// k % d).  The (term, coordinate) pair is walked forward from the lane's
// first k rather than divided out per element.  Rows past np are zero.
template <int SPLIT, int KS, typename T>
__device__ __forceinline__ void write_a_operands(const T* X, int p0, int np, int d, int XS,
                                                 const float* xs, u16x8* Apre) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int row = w * 16 + (lane % 16);
  const bool valid = row < np;
  int part = 0, coord = (lane / 16) * 8;
  while (coord >= d) {
    coord -= d;
    ++part;
  }
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    u16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      v[e] = (valid && part < SPLIT)
                 ? a_elem<SPLIT>(op_elem<T>(X, (int64_t)(p0 + row) * d + coord, xs[row * XS + coord]), part)
                 : (uint16_t)0;
      if (++coord == d) {
        coord = 0;
        ++part;
      }
    }
    if (s + 1 < KS) {  // on to k = (s + 1) * 32 + (lane / 16) * 8
      coord += 24;
      while (coord >= d) {
        coord -= d;
        ++part;
      }
    }
    Apre[((int64_t)(p0 / 16 + w) * KS + s) * 64 + lane] = v;
  }
}

// The point side of the screen, built once per call: the A operands above
// for every tile of 16 points, and ||x||^2 when norms != nullptr.  Rows are
// staged through LDS as FP32 with coalesced loads.  Tiles past n are zero.
// Without PREP only the norms are written.
template <int SPLIT, int KS, typename T, bool PREP>
__global__ __launch_bounds__(256) void k_prep_a(const T* X, const float* row_scale, int n, int d,
                                                float* norms, u16x8* Apre) {
  extern __shared__ float xs[];  // [64][XS], XS = d + 1 when d is a multiple of 32
  __shared__ float ss[64];       // FP8 row scales
  const int pad = d % 32 == 0 ? 1 : 0, XS = d + pad;
  const int p0 = blockIdx.x * 64;
  const int np = max(0, min(64, n - p0));
  stage_rows<T>(X, row_scale, p0, np, d, pad, ss, xs);
  __syncthreads();
  if (norms && threadIdx.x < np) norms[p0 + threadIdx.x] = staged_norm(xs + threadIdx.x * XS, d);
  if constexpr (PREP) write_a_operands<SPLIT, KS, T>(X, p0, np, d, XS, xs, Apre);
}

// ------------------------------------------------------------ first pass
// Algorithm 2 step 2 (the first pass, m = 1) fused with the preparation of
// the A operands: one coalesced read of each block of 64 rows of X gives
// D^2 to the first center (FP32 direct form, coordinates ascending, as the
// fold computes it), A = its id, ||x||^2 (when norms != nullptr) and, when
// PREP, the A operands exactly as k_prep_a writes them.
template <int SPLIT, int KS, typename T, bool PREP>
__global__ __launch_bounds__(256) void k_first_prep(const T* X, const float* row_scale, int n,
                                                    int d, int DP, const float* C, const int* rs,
                                                    float* D2, int* A, float* norms,
                                                    u16x8* Apre) {
  // [64][XS] rows, then the first center [DP]; XS = d + 1 when d is a
  // multiple of 32, so the 64 threads that walk one row each do not all read
  // the same bank
  extern __shared__ float xs[];
  __shared__ float ss[64];       // FP8 row scales
  const int pad = d % 32 == 0 ? 1 : 0, XS = d + pad;
  float* c0 = xs + 64 * XS;
  const int p0 = blockIdx.x * 64;
  const int np = max(0, min(64, n - p0));
  const int id0 = rs[0];
  for (int e = threadIdx.x; e < DP; e += 256) c0[e] = C[(int64_t)id0 * DP + e];
  stage_rows<T>(X, row_scale, p0, np, d, pad, ss, xs);
  __syncthreads();
  if (threadIdx.x < np) {
    const float* xr = xs + threadIdx.x * XS;
    float acc = 0.0f, nx = 0.0f;
#pragma unroll 8
    for (int e = 0; e < d; ++e) {
      const float v = xr[e];
      const float t = v - c0[e];
      acc = fmaf(t, t, acc);
      nx = fmaf(v, v, nx);
    }
    const int i = p0 + threadIdx.x;
    if (norms) norms[i] = nx;
    D2[i] = acc;
    A[i] = id0;
  }
  if constexpr (PREP) write_a_operands<SPLIT, KS, T>(X, p0, np, d, XS, xs, Apre);
}

// --------------------------------------------------------------- the screen
// Block = kWaves waves; wave w owns KRT tiles of 16 points (A operands held in
// registers for the pass).  Candidate tiles stream through two LDS buffers:
// while the waves compute on chunk c, the direct global->LDS loads of chunk
// c+1 are in flight.  Each accumulator starts at -ncg_j/2, so it ends as
// acc = x.c - ncg_j/2 = -(lb - (1-2G)||x||^2)/2, and the smallest lb is the
// largest acc.
template <int KS, typename T>
constexpr int screen_krt_t() {
  return screen_krt(KS, ScaledRows<T>::value);
}

typedef __attribute__((address_space(3))) void lds_void;
typedef const __attribute__((address_space(1))) void gbl_void;

// acc[r] = A[r] . B(tile q) - ncg_j / 2, for the wave's KRT row tiles
// (SC: acc[r] = A[r] . B(tile q); the epilogue scales and biases it).
template <int KS, int KRT, bool BCAST, bool SC>
__device__ __forceinline__ void mfma_tile(const bf16x8 (&Aop)[KRT][KS], const u16x8* buf,
                                          const float* ncs, int q, int lane, f32x4 (&acc)[KRT]) {
  // ncs: -ncg/2 per candidate, four copies each when BCAST (one LDS read
  // then yields the accumulator's initial value)
  f32x4 cinit;
  if constexpr (SC) {
    cinit = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  } else if constexpr (BCAST) {
    cinit = reinterpret_cast<const f32x4*>(ncs)[q * 16 + (lane % 16)];
  } else {
    const float cj = ncs[q * 16 + (lane % 16)];
    cinit = f32x4{cj, cj, cj, cj};
  }
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const bf16x8 b = __builtin_bit_cast(bf16x8, buf[(q * KS + s) * 64 + lane]);
#pragma unroll
    for (int r = 0; r < KRT; ++r)
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop[r][s], b, s == 0 ? cinit : acc[r], 0, 0, 0);
  }
}

// Largest and second largest tagged acc of each (row tile, row): the low
// bits of each value are replaced by the tile's position tq first.  Tagged
// values are finite, so med3 with FLT_MAX is their max, without the quieting
// moves fmaxf would add.  SC: each value is first scaled and biased,
// acc * (s_row * s_j) - ncg_j / 2, with (-ncg_j / 2, s_j) of tile q's column
// j from ncs and the row scales srow.
template <int KRT, bool SC>
__device__ __forceinline__ void epilogue(const f32x4 (&acc)[KRT], uint32_t keep, uint32_t tq,
                                         float (&s1)[KRT][4], float (&s2)[KRT][4],
                                         const float (&srow)[KRT][4], const float* ncs, int q,
                                         int lane, unsigned skip = 0) {
  float2 col = make_float2(0.0f, 0.0f);
  if constexpr (SC) col = reinterpret_cast<const float2*>(ncs)[q * 16 + (lane % 16)];
#pragma unroll
  for (int r = 0; r < KRT; ++r) {
    if ((skip >> r) & 1u) continue;  // row tile r cannot gain from this tile (wave-uniform)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float a = acc[r][i];
      if constexpr (SC) a = fmaf(a, srow[r][i] * col.y, col.x);
      const float v = __uint_as_float((__float_as_uint(a) & keep) | tq);
      s2[r][i] = __builtin_amdgcn_fmed3f(s1[r][i], s2[r][i], v);
      s1[r][i] = __builtin_amdgcn_fmed3f(s1[r][i], v, FLT_MAX);
    }
  }
}

// Starts the copy of rows [row0, row0 + nr) of X (raw elements, rowb bytes
// each, nr * rowb a multiple of 16) straight from global memory into dst:
// lane i of each 1 KB step lands at dst + v0 + 16 i.  The copy is complete
// after the next vmcnt(0) wait.
template <typename T>
__device__ __forceinline__ void stage_rows(char* dst, const T* X, int64_t row0, int nr, int rowb,
                                           int lane) {
  const int bytes = nr * rowb;
  const char* src = reinterpret_cast<const char*>(X) + row0 * rowb;
  for (int v0 = 0; v0 < bytes; v0 += 1024)
    if (v0 + 16 * lane < bytes)
      __builtin_amdgcn_global_load_lds((gbl_void*)(src + v0 + 16 * lane), (lds_void*)(dst + v0),
                                       16, 0, 0);
}

// FP32 direct form sum_e (x_e - c_e)^2, e ascending, exactly as the plain
// kernels compute it (the terms past d add fmaf(0, 0, r) = r).  x: a raw
// row (decoded with the row scale sc), staged in LDS (XLDS: read 32 elements
// at a time without guards; reads past the row stay inside LDS) or in X
// (guarded); c: an FP32 candidate row (16-byte aligned), read eight float4
// at a time.
template <typename T, bool XLDS>
__device__ __forceinline__ float refine_dist(const T* x, const float* c, int d, float sc) {
  float r = 0.0f;
  for (int e0 = 0; e0 < d; e0 += 32) {
    float4 cv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      cv[u] = (e0 + 4 * u < d) ? reinterpret_cast<const float4*>(c + e0)[u]
                               : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float xv[32];
#pragma unroll
    for (int k = 0; k < 32; ++k)
      xv[k] = (XLDS || e0 + k < d) ? Elem<T>::get(x, e0 + k, sc) : 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float cc[4] = {cv[u].x, cv[u].y, cv[u].z, cv[u].w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + 4 * u + q;
        const float t = e < d ? xv[4 * u + q] - cc[q] : 0.0f;
        r = fmaf(t, t, r);
      }
    }
  }
  return r;
}

// The screen of block `blk` of the points of `a` (kWaves * KRT * 16 points).
// ONEG: the pass has at most kScreenOneGroupMaxTiles tiles and each value
// carries its tile's index in the pass (a.tag_bits bits), so the running
// maxima are the pass's maxima and no per-group maxima or ids are kept.
template <int SPLIT, int KS, typename T, bool DIRECT, bool ONEG, bool PRUNE = false>
__device__ __forceinline__ void screen_body(const ScreenArgs& a, int blk) {
  constexpr int KRT = screen_krt_t<KS, T>();  // row tiles per wave
  constexpr int WP = KRT * 16;         // points per wave
  constexpr int BP = kWaves * WP;      // points per block
  // the single-group screen of up to four k-steps of unscaled rows runs
  // three waves per SIMD (smaller staging, no software pipeline)
  constexpr bool THREE = screen_three_waves(KS, ONEG, ScaledRows<T>::value);
  constexpr bool PIPE = !THREE;
  constexpr bool SCR = ScaledRows<T>::value;
  constexpr int STAGE = screen_stage_bytes(KS, ONEG, SCR);  // bytes per staging buffer
  constexpr int WSTAGE = screen_wave_stage(KS, ONEG, SCR);  // a wave's share after the pass
  constexpr int CT = screen_chunk_tiles(KS, ONEG, SCR);     // candidate tiles per chunk
  static_assert(CT >= 1 && CT * KS * 64 * 16 <= STAGE, "chunk exceeds its staging buffer");
  constexpr int CHUNK_V = CT * KS * 64;             // 16-byte vectors per chunk
  // Two full staging buffers whatever the chunk: after the pass each wave
  // reuses a quarter of them (WSTAGE bytes) for its own data.  They are two
  // distinct arrays, and each chunk reads one named array while the direct
  // loads fill the other: the compiler then knows that the chunk's LDS reads
  // do not alias the loads in flight and does not wait for them.
  __shared__ u16x8 sB0[STAGE / 16];
  __shared__ u16x8 sB1[STAGE / 16];
  static_assert(2 * STAGE == kWaves * WSTAGE, "wave quarters must tile the buffers");
  constexpr bool SC = ScaledRows<T>::value;  // codes with row scales
  constexpr bool BCAST = screen_bcast(KS, ONEG, SC);  // LDS for four copies of each bias
  // per candidate: -ncg/2 (four copies when BCAST), or (-ncg/2, scale) when SC
  __shared__ __attribute__((aligned(16))) float sN[2][CT * 16 * (BCAST ? 4 : (SC ? 2 : 1))];

  // the wave index is uniform across the wave: kept in a scalar register, it
  // makes the chunk staging loop a scalar loop
  const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int d = a.d;
  int id0 = a.id0_host, m = a.m_host;
  if (a.rs) {
    id0 = a.rs[0];
    m = a.rs[1] - id0;
  }
  const int ntiles = (m + 15) / 16;
  const int nchunks = (ntiles + CT - 1) / CT;
  const int wbase = blk * BP + wave * WP;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const u16x8* __restrict__ Bg = static_cast<const u16x8*>(a.B);

  // Issues the direct loads of chunk c into dst (each wave moves 1 KB per
  // instruction; lane i lands at base + 16 i).
  auto stage = [&](int c, u16x8* dst) __attribute__((always_inline)) {
    const int nt = min(CT, ntiles - c * CT);
    const int nv = nt * KS * 64;
    const u16x8* src = Bg + (int64_t)c * CHUNK_V;
    for (int v0 = wave * 64; v0 < nv; v0 += kWaves * 64)
      __builtin_amdgcn_global_load_lds((gbl_void*)(src + v0 + lane), (lds_void*)(dst + v0), 16, 0, 0);
  };
  // A chunk's CT * 16 biases, NBT per thread (two when a chunk holds 32
  // tiles, i.e. KS = 1).
  constexpr int NBT = (CT * 16 + kWaves * 64 - 1) / (kWaves * 64);
  float ncg_next[NBT], scg_next[NBT];
  auto stage_ncg = [&](int c) {
#pragma unroll
    for (int i = 0; i < NBT; ++i) {
      const int e = i * kWaves * 64 + threadIdx.x;  // bias within the chunk
      const int idx = c * CT * 16 + e;
      const bool in = e < CT * 16 && idx < ntiles * 16;
      ncg_next[i] = in ? a.ncg[idx] : INFINITY;
      if constexpr (SC) scg_next[i] = in ? a.scg[idx] : 0.0f;
    }
  };

  // Tile skip (three-wave single-group screen of a pass that keeps D):
  // ||x - c||^2 >= (||x|| - ||c||)^2, so a candidate tile whose norm
  // interval lies far enough from a row tile's cannot bring any of its
  // points below D (nor within the band of it).  Lane j < CT * KRT judges
  // (tile j / KRT of a chunk, row tile j % KRT).
  static_assert(!PRUNE || THREE, "the tile skip is built into the three-wave screen only");
  const bool prune = PRUNE && a.tnr != nullptr && !a.first;
  float2 tnr_next = make_float2(INFINITY, 0.0f);
  auto stage_tnr = [&](int c) {
    const int tq = c * CT + lane / KRT;
    tnr_next = (prune && lane < CT * KRT && tq < ntiles) ? a.tnr[tq] : make_float2(INFINITY, 0.0f);
  };
  if (nchunks > 0) stage(0, sB0);
  stage_ncg(0);
  stage_tnr(0);
  unsigned folded = 0;  // tile skip: bit r, row tile r took the values of some tile

  // A operands of this wave's points, kept in registers for the pass: from
  // the prepared buffer, or straight from X when d % 8 == 0 and X is bf16
  // (its rows then already hold the operand bytes) or FP8 (eight codes per
  // lane and k-step, converted exactly; part p of the K axis is the row).
  bf16x8 Aop[KRT][KS];
#pragma unroll
  for (int r = 0; r < KRT; ++r) {
    const int tile = wbase / 16 + r;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
      if constexpr (DIRECT) {
        const int p = wbase + r * 16 + (lane % 16);
        const int k0 = s * 32 + (lane / 16) * 8;
        const int part = k0 / d, coord = k0 - part * d;
        if (p < a.n && part < SPLIT) {
          if constexpr (SC) {
            const uint2 w = *reinterpret_cast<const uint2*>(
                reinterpret_cast<const uint8_t*>(a.X) + (int64_t)p * d + coord);
#pragma unroll
            for (int e = 0; e < 8; ++e)
              v[e] = code_bf16((uint8_t)((e < 4 ? w.x : w.y) >> (8 * (e % 4))));
          } else {
            v = *reinterpret_cast<const u16x8*>(static_cast<const uint16_t*>(a.X) + (int64_t)p * d + coord);
          }
        }
      } else {
        v = static_cast<const u16x8*>(a.Apre)[((int64_t)tile * KS + s) * 64 + lane];
      }
      Aop[r][s] = __builtin_bit_cast(bf16x8, v);
    }
  }

  // Per tag group, the largest and second largest tagged acc of each (row
  // tile, row), the tag being the tile's position in the group; after each
  // group they are merged into the running largest, second largest and
  // argmax.  ONEG: one group, the whole pass, folded straight into the
  // running pair.  The mask lives in a VGPR so that the tag insert is one
  // v_and_or_b32 (VOP3 reads at most one SGPR, and the tile position is one).
  constexpr int GC = ONEG ? 1 << 20 : screen_group_chunks(KS);  // chunks per tag group
  constexpr int TBG = screen_tag_bits(KS);
  static_assert(ONEG || (1 << TBG) >= screen_group_chunks(KS) * CT, "tag too narrow for a group");
  const int TB = ONEG ? a.tag_bits : TBG;
  // a pass with more tiles than the tag can number (the host sizes the tag
  // from the pass's capacity) is left to the direct form
  const bool tag_ok = !ONEG || (TB >= 1 && TB <= 10 && ntiles <= (1 << TB));
  uint32_t keep;
  asm volatile("v_mov_b32 %0, %1" : "=v"(keep) : "s"(~((1u << TB) - 1u)));
  // SC: the scales of the rows of each value (0 outside the screen's range:
  // such a point is listed whatever its values)
  float srow[KRT][4];
#pragma unroll
  for (int r = 0; r < KRT; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      srow[r][i] = 0.0f;
      if constexpr (SC) {
        const int p = wbase + r * 16 + (lane / 16) * 4 + i;
        const float sp = p < a.n ? a.row_scale[p] : 0.0f;
        srow[r][i] = (sp >= kScaleMin && sp <= kScaleMax) ? sp : 0.0f;
      }
    }
  // The norm interval [xlo, xhi] and the distance limit dlim of row tile
  // lane % KRT (reduced over its 16 points), for the tile skip.  ||x||
  // comes from the FP32 ||x||^2 (relative error below (d + 1) 2^-24 before
  // the root), widened by (d + 8) 2^-24; a point without finite norm or D
  // keeps its row tile from being skipped.
  float pxlo = INFINITY, pxhi = 0.0f, pdl = 0.0f;
  if (prune) {
    const float ue = 0x1.0p-24f;
    const int pl = wbase + lane;
    float xl = INFINITY, xh = 0.0f, dl = 0.0f;
    if (lane < WP && pl < a.n) {
      const float n2 = a.norms[pl], dd = a.D2[pl];
      if (n2 >= 0.0f && n2 <= FLT_MAX && dd >= 0.0f && dd <= FLT_MAX) {
        const float x = sqrtf(n2);
        xl = x * (1.0f - (d + 8) * ue);
        xh = x * (1.0f + (d + 8) * ue);
        dl = dd;
      } else {
        xl = 0.0f;
        xh = INFINITY;
        dl = INFINITY;
      }
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      xl = fminf(xl, __shfl_xor(xl, off, 16));
      xh = fmaxf(xh, __shfl_xor(xh, off, 16));
      dl = fmaxf(dl, __shfl_xor(dl, off, 16));
    }
    const int src = 16 * (lane % KRT);
    pxlo = __shfl(xl, src);
    pxhi = __shfl(xh, src);
    // a skipped candidate must lie beyond (1 + 2 band) D in the FP32 direct
    // form, band = 2 (d + 2) 2^-24: D is raised and the squared gap lowered
    // by more than that and every rounding of the test
    pdl = __shfl(dl, src) * (1.0f + (8 * d + 32) * ue);
  }
  float s1[KRT][4], s2[KRT][4], c1[KRT][4], c2[KRT][4];
  int ix[KRT][4];
#pragma unroll
  for (int r = 0; r < KRT; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s1[r][i] = -INFINITY;
      s2[r][i] = -INFINITY;
      ix[r][i] = -1;
    }

  // Chunk c, held in buf (sB0 for even c, sB1 for odd c); chunk c + 1 goes
  // to next.
  auto chunk = [&](int c, const u16x8* buf, u16x8* next) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NBT; ++i) {
      const int e = i * kWaves * 64 + threadIdx.x;
      if (e < CT * 16) {
        const float nb = -0.5f * fminf(ncg_next[i], FLT_MAX);
        if constexpr (SC)
          reinterpret_cast<float2*>(sN[c & 1])[e] = make_float2(nb, scg_next[i]);
        else if constexpr (BCAST)
          reinterpret_cast<f32x4*>(sN[c & 1])[e] = f32x4{nb, nb, nb, nb};
        else
          sN[c & 1][e] = nb;
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();  // chunk c is in LDS; everyone is done with chunk c-1
    // bit q * KRT + r: row tile r skips tile q of this chunk
    uint64_t skipm = 0;
    if (prune) {
      const float gap = fmaxf(tnr_next.x - pxhi, pxlo - tnr_next.y);
      const float ue = 0x1.0p-24f;
      skipm = __ballot(gap > 0.0f && gap * gap * (1.0f - (2 * d + 16) * ue) > pdl);
    }
    if (c + 1 < nchunks) {
      stage(c + 1, next);
      stage_ncg(c + 1);
      stage_tnr(c + 1);
    }
    const int nt = min(CT, ntiles - c * CT);
    const float* ncs = sN[c & 1];
    const int cg = ONEG ? c : c % GC;  // position of the chunk in its tag group
    const uint32_t t0 = cg * CT;       // tag of the chunk's first tile
    if (!ONEG && cg == 0) {
#pragma unroll
      for (int r = 0; r < KRT; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          c1[r][i] = -INFINITY;
          c2[r][i] = -INFINITY;
        }
    }
    // Software pipeline: the MFMAs of tile q+1 are issued before the
    // epilogue of tile q, so matrix and vector units overlap within a wave
    // (two accumulator sets, unrolled by two so no copies are needed).
    f32x4 acc0[KRT], acc1[KRT];
    // each tile's values go to the group pair (the running pair when ONEG)
    auto fold = [&](const f32x4 (&acc)[KRT], int q, unsigned sk = 0) {
      if constexpr (ONEG)
        epilogue<KRT, SC>(acc, keep, t0 + q, s1, s2, srow, ncs, q, lane, sk);
      else
        epilogue<KRT, SC>(acc, keep, t0 + q, c1, c2, srow, ncs, q, lane, sk);
    };
    if constexpr (!PIPE) {
      // three waves per SIMD: the other waves' vector work overlaps a
      // wave's matrix instructions, so one accumulator set suffices
      constexpr unsigned FULL = (1u << KRT) - 1u;
      for (int q = 0; q < nt; ++q) {
        // a chunk of more than 64 / KRT tiles (one k-step) has judges for
        // its first 64 / KRT tiles only; the rest are never skipped
        const unsigned sk = q * KRT < 64 ? (unsigned)(skipm >> (q * KRT)) & FULL : 0u;
        if (sk == FULL) continue;  // no row tile of the wave can gain from tile q
        folded |= ~sk & FULL;
        mfma_tile<KS, KRT, BCAST, SC>(Aop, buf, ncs, q, lane, acc0);
        fold(acc0, q, sk);
      }
    } else {
    mfma_tile<KS, KRT, BCAST, SC>(Aop, buf, ncs, 0, lane, acc0);
    int q = 0;
    for (; q + 2 < nt; q += 2) {
      mfma_tile<KS, KRT, BCAST, SC>(Aop, buf, ncs, q + 1, lane, acc1);
      fold(acc0, q);
      mfma_tile<KS, KRT, BCAST, SC>(Aop, buf, ncs, q + 2, lane, acc0);
      fold(acc1, q + 1);
      // Issue order: the operand reads first, then every MFMA followed by
      // three vector instructions, so that one wave keeps both the matrix
      // and the vector pipes busy.
      __builtin_amdgcn_sched_group_barrier(0x100, 2 * (KS + 1), 0);
#pragma unroll
      for (int g = 0; g < 2 * KS * KRT; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
      }
    }
    if (q + 1 < nt) {
      mfma_tile<KS, KRT, BCAST, SC>(Aop, buf, ncs, q + 1, lane, acc1);
      fold(acc0, q);
      fold(acc1, q + 1);
    } else {
      fold(acc0, q);
    }
    }
    // Group merge: candidate id from the tag and the lane's column; a tie
    // with the running maximum keeps the earlier (lower) id.
    if (!ONEG && (cg == GC - 1 || c + 1 == nchunks)) {
#pragma unroll
    for (int r = 0; r < KRT; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v1 = c1[r][i];
        const int cj = ((int)(__float_as_uint(v1) & ((1u << TB) - 1u)) + (c - cg) * CT) * 16 + (lane % 16);
        const bool take = v1 > s1[r][i];
        s2[r][i] = __builtin_amdgcn_fmed3f(s1[r][i], v1,
                                           __builtin_amdgcn_fmed3f(s2[r][i], c2[r][i], FLT_MAX));
        ix[r][i] = take ? cj : ix[r][i];
        s1[r][i] = __builtin_amdgcn_fmed3f(s1[r][i], v1, FLT_MAX);
      }
    }
  };
  for (int c = 0; c < nchunks; c += 2) {
    chunk(c, sB0, sB1);
    if (c + 1 < nchunks) chunk(c + 1, sB1, sB0);
  }

  // Once every wave is past its last chunk the staging buffers are idle and
  // each wave works in its own quarter of them (waves 0 and 1 in sB0, 2 and
  // 3 in sB1).
  __syncthreads();
  const int p = wbase + lane;
  const bool valid = lane < WP && p < a.n;  // lanes past the wave's points idle
  const float nx = valid ? a.norms[p] : 0.0f;
  const float D = (a.first || !valid) ? INFINITY : a.D2[p];
  static_assert(2 * WSTAGE == STAGE, "two wave quarters per staging buffer");
  char* xw = reinterpret_cast<char*>(wave < 2 ? sB0 : sB1) + (wave & 1) * WSTAGE;

  // Merge of the 16 columns of every point through LDS: lane l writes the
  // (largest, second largest, id) of each (row tile, row) at [point][l % 16]
  // (columns XOR-swizzled by the point to spread the banks), then lane p
  // reads the 16 entries of point p and merges them in column order.  Of two
  // equal maxima the earlier column is kept; no decision depends on which,
  // since then lb2 = lbmin <= r1 and the point is listed.  When the wave's
  // share cannot hold all its points' entries, the points go in two halves.
  // ONEG: a maximum's id is its tag (tile index in the pass) and the column.
  constexpr int HALVES = WP * 16 * 16 > WSTAGE ? 2 : 1;
  constexpr int PH = WP / HALVES;  // points per half
  static_assert(PH * 16 * 16 <= WSTAGE && PH % 16 == 0, "merge exceeds the wave's share");
  f32x4* M = reinterpret_cast<f32x4*>(xw);  // [PH points][16 columns]
  float b1 = -INFINITY, b2 = -INFINITY;
  int j1 = -1;
#pragma unroll
  for (int h = 0; h < HALVES; ++h) {
#pragma unroll
    for (int r = h * (KRT / HALVES); r < (h + 1) * (KRT / HALVES); ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pl = r * 16 + (lane / 16) * 4 + i - h * PH;
        int id;
        if constexpr (ONEG)
          id = (int)(__float_as_uint(s1[r][i]) & ~keep) * 16 + (lane % 16);
        else
          id = ix[r][i];
        M[pl * 16 + ((lane % 16) ^ (pl & 15))] = f32x4{s1[r][i], s2[r][i], __int_as_float(id), 0.0f};
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane / PH == h) {  // this lane's point is in the half
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const f32x4 e = M[(lane - h * PH) * 16 + (c ^ (lane & 15))];
        const bool take = e.x > b1;
        b2 = __builtin_amdgcn_fmed3f(b1, e.x, __builtin_amdgcn_fmed3f(b2, e.y, FLT_MAX));
        j1 = take ? __float_as_int(e.z) : j1;
        b1 = __builtin_amdgcn_fmed3f(b1, e.x, FLT_MAX);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the share is free again
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }

  // This wave's rows (raw elements) go to its quarter: full waves stage them
  // in groups of R (a multiple of 16, so every group is whole 16-byte units);
  // the one partial wave of X reads its rows from global memory instead.
  const int nvalid = max(0, min(WP, a.n - wbase));
  const int rowb = d * (int)sizeof(T);  // <= 1 KB, so R >= 16
  const int R = min(WP, (WSTAGE / rowb) & ~15);  // rows per staging group

  // One lane per point: decide, refine, fold or list.  The refinement
  // reads the point's row (from a staged copy, or from X) and the candidate
  // row as float4.
  float sp = 1.0f;  // the point's row scale (FP8)
  if constexpr (SC) sp = valid ? a.row_scale[p] : 0.0f;
  const bool in_range = tag_ok && nx >= kNormMin && nx <= kNormMax &&
                        (!SC || (sp >= kScaleMin && sp <= kScaleMax));
  const float nxg = a.oneminus2g * nx;
  const float lbmin = fmaf(b1, -2.0f, nxg);
  const float lb2 = fmaf(b2, -2.0f, nxg);
  const bool jok = j1 >= 0 && j1 < m;  // a candidate of the pass, not a padding column
  // the winner's candidate: tiles hold the candidates in norm order when
  // the pass sorted them (cperm), else in id order
  const int jc = (jok && a.cperm) ? a.cperm[j1] : j1;
  const bool refine = valid && in_range && jok && lbmin < D;
  const float* crow = a.C + (int64_t)(id0 + (jok ? jc : 0)) * a.DP;  // read only when refining
  // A full wave copies its rows into LDS (one coalesced copy) unless none of
  // its lanes refines.
  const bool staged = nvalid == WP && __ballot(refine) != 0;
  if (staged) stage_rows<T>(xw, X, wbase, R, rowb, lane);
  float r1 = 0.0f;
  if (staged) {
    for (int c0 = 0; c0 < WP; c0 += R) {
      const int nr = min(R, WP - c0);
      if (c0 > 0) {
        __builtin_amdgcn_wave_barrier();  // the previous group has been read
        stage_rows<T>(xw, X, wbase + c0, nr, rowb, lane);
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __builtin_amdgcn_wave_barrier();
      if (refine && lane >= c0 && lane < c0 + nr)
        r1 = refine_dist<T, true>(reinterpret_cast<const T*>(xw + (lane - c0) * rowb), crow, d, sp);
    }
  } else if (refine) {
    r1 = refine_dist<T, false>(X + (int64_t)p * d, crow, d, sp);
  }
  if (!valid) return;
  // S (when kept), the second-smallest distance, is exact wherever it is at
  // most (1 + band) D2 with band = 2 (d + 2) 2^-24: a bound lb of a
  // candidate sits at least G S_c below its distance, G >= 2 band, so a
  // candidate certified by lb >= D (or lb2 > r1) lies beyond that and leaves
  // S's near-tie status as it was.
  bool listed = false;
  if (!in_range) {
    // outside the bound's range: the direct form decides (points already at
    // zero distance too when S is kept, for a tie at zero)
    listed = D > 0.0f || a.S != nullptr;
  } else if (!refine) {
    // lbmin >= D: no candidate comes closer.  Without a usable winner (only
    // non-finite values give none) or in a first pass, which writes every
    // point, the direct form decides.
    if (!a.first && jok && lbmin >= D) return;
    // The tile skip ruled out every tile of the pass for this point's row
    // tile: each candidate lies beyond the band above D, so D, A and S stand.
    if (prune && nchunks > 0 && !((folded >> (lane / 16)) & 1u)) return;
    listed = true;
  } else if (r1 < D) {
    if (lb2 > r1) {
      if (a.S) a.S[p] = D;
      a.D2[p] = r1;
      a.A[p] = id0 + jc;
    } else {
      listed = true;
    }
  } else if (!(lb2 >= D)) {
    listed = true;
  } else if (a.S) {
    a.S[p] = fminf(a.S[p], r1);
  }
  if (listed) {
    const int pos = atomicAdd(a.list_len, 1);
    a.list[pos] = p;
  }
}

// The grouped screen runs two waves per SIMD up to six k-steps (one beyond).
template <int SPLIT, int KS, typename T, bool DIRECT>
__global__ __launch_bounds__(kWaves * 64) __attribute__((amdgpu_waves_per_eu(KS <= 6 ? 2 : 1)))
void k_screen(ScreenArgs a) {
  screen_body<SPLIT, KS, T, DIRECT, false>(a, blockIdx.x);
}
// The single-group screen; k_screen_one3, held to the registers of three
// waves per SIMD, where its shape runs three (screen_three_waves).
template <int SPLIT, int KS, typename T, bool DIRECT>
__global__ __launch_bounds__(kWaves * 64) void k_screen_one(ScreenArgs a) {
  screen_body<SPLIT, KS, T, DIRECT, true>(a, blockIdx.x);
}
template <int SPLIT, int KS, typename T, bool DIRECT, bool PRUNE>
__global__ __launch_bounds__(kWaves * 64) __attribute__((amdgpu_waves_per_eu(3)))
void k_screen_one3(ScreenArgs a) {
  screen_body<SPLIT, KS, T, DIRECT, true, PRUNE>(a, blockIdx.x);
}

// Adds the previous pass's listed count to the stats and clears it.
__global__ void k_list_reset(int* list_len, kmpar_stats* st) {
  if (threadIdx.x == 0) {
    if (st) st->n_rescanned += *list_len;
    *list_len = 0;
  }
}

template <int SPLIT, int KS, typename T>
static void launch_one(const ScreenArgs& a, hipStream_t s) {
  constexpr int BP = kWaves * screen_krt_t<KS, T>() * 16;
  const int blocks = (a.n + BP - 1) / BP;
  constexpr bool THREE = screen_three_waves(KS, true, ScaledRows<T>::value);
  if (a.tag_bits > 0) {
    if constexpr (THREE) {
      // passes that keep D with sorted candidate tiles take the tile skip
      const bool pr = a.tnr != nullptr && !a.first;
      if (a.Apre && pr)
        hipLaunchKernelGGL((k_screen_one3<SPLIT, KS, T, false, true>), dim3(blocks), dim3(kWaves * 64), 0, s, a);
      else if (a.Apre)
        hipLaunchKernelGGL((k_screen_one3<SPLIT, KS, T, false, false>), dim3(blocks), dim3(kWaves * 64), 0, s, a);
      else if (pr)
        hipLaunchKernelGGL((k_screen_one3<SPLIT, KS, T, true, true>), dim3(blocks), dim3(kWaves * 64), 0, s, a);
      else
        hipLaunchKernelGGL((k_screen_one3<SPLIT, KS, T, true, false>), dim3(blocks), dim3(kWaves * 64), 0, s, a);
    } else {
      if (a.Apre)
        hipLaunchKernelGGL((k_screen_one<SPLIT, KS, T, false>), dim3(blocks), dim3(kWaves * 64), 0, s, a);
      else
        hipLaunchKernelGGL((k_screen_one<SPLIT, KS, T, true>), dim3(blocks), dim3(kWaves * 64), 0, s, a);
    }
  } else if (a.Apre) {
    hipLaunchKernelGGL((k_screen<SPLIT, KS, T, false>), dim3(blocks), dim3(kWaves * 64), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_screen<SPLIT, KS, T, true>), dim3(blocks), dim3(kWaves * 64), 0, s, a);
  }
}

// KS k-steps, dispatched up to MAXKS (the widest row the dtype and split
// can have).
template <int SPLIT, typename T, int MAXKS = kScreenMaxKS>
static hipError_t launch_split(int KS, const ScreenArgs& a, hipStream_t s) {
  if (KS < 1 || KS > MAXKS) return hipErrorInvalidValue;
  switch (KS) {
#define KMPAR_LS(V) \
  case V: if constexpr (V <= MAXKS) launch_one<SPLIT, V, T>(a, s); break;
    KMPAR_LS(1) KMPAR_LS(2) KMPAR_LS(3) KMPAR_LS(4) KMPAR_LS(5) KMPAR_LS(6) KMPAR_LS(7)
    KMPAR_LS(8) KMPAR_LS(9) KMPAR_LS(10) KMPAR_LS(11) KMPAR_LS(12) KMPAR_LS(13) KMPAR_LS(14)
    KMPAR_LS(15) KMPAR_LS(16)
#undef KMPAR_LS
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// PREP: A operands for every 256-point block (tiles past n zero) plus the
// norms; otherwise the norms alone, one block per 64 rows.
template <int SPLIT, int KS, typename T, bool PREP = true>
static hipError_t launch_prep_a_one(const void* X, const float* rsc, int n, int d, float* norms,
                                    void* Apre, hipStream_t s) {
  const int blocks = PREP ? (n + kBlockPts - 1) / kBlockPts * (kBlockPts / 64) : (n + 63) / 64;
  const size_t lds = (size_t)64 * (d + (d % 32 == 0 ? 1 : 0)) * 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_prep_a<SPLIT, KS, T, PREP>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_prep_a<SPLIT, KS, T, PREP>), dim3(blocks), dim3(256), lds, s,
                     static_cast<const T*>(X), rsc, n, d, norms, static_cast<u16x8*>(Apre));
  return hipGetLastError();
}

template <int SPLIT, typename T, int MAXKS = kScreenMaxKS>
static hipError_t launch_prep_a_split(int KS, const void* X, const float* rsc, int n, int d,
                                      float* norms, void* Apre, hipStream_t s) {
  if (KS < 1 || KS > MAXKS) return hipErrorInvalidValue;
  switch (KS) {
#define KMPAR_PA(V) \
  case V: if constexpr (V <= MAXKS) return launch_prep_a_one<SPLIT, V, T>(X, rsc, n, d, norms, Apre, s); break;
    KMPAR_PA(1) KMPAR_PA(2) KMPAR_PA(3) KMPAR_PA(4) KMPAR_PA(5) KMPAR_PA(6) KMPAR_PA(7)
    KMPAR_PA(8) KMPAR_PA(9) KMPAR_PA(10) KMPAR_PA(11) KMPAR_PA(12) KMPAR_PA(13) KMPAR_PA(14)
    KMPAR_PA(15) KMPAR_PA(16)
#undef KMPAR_PA
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int SPLIT, int KS, typename T, bool PREP>
static hipError_t launch_first_one(const void* X, const float* rsc, int n, int d, int DP,
                                   const float* C, const int* rs, float* D2, int* A,
                                   float* norms, void* Apre, hipStream_t s) {
  // grid: 64-row blocks; with PREP the A tiles of all ceil(n / 256) * 16
  // tiles the screen reads are written (rows past n as zeros)
  const int blocks = PREP ? (n + kBlockPts - 1) / kBlockPts * (kBlockPts / 64) : (n + 63) / 64;
  const size_t lds = ((size_t)64 * (d + (d % 32 == 0 ? 1 : 0)) + DP) * 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_first_prep<SPLIT, KS, T, PREP>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_first_prep<SPLIT, KS, T, PREP>), dim3(blocks), dim3(256), lds, s,
                     static_cast<const T*>(X), rsc, n, d, DP, C, rs, D2, A, norms,
                     static_cast<u16x8*>(Apre));
  return hipGetLastError();
}

template <int SPLIT, typename T, int MAXKS = kScreenMaxKS>
static hipError_t launch_first_split(int KS, const void* X, const float* rsc, int n, int d, int DP,
                                     const float* C, const int* rs, float* D2, int* A,
                                     float* norms, void* Apre, hipStream_t s) {
  if (KS < 1 || KS > MAXKS) return hipErrorInvalidValue;
  switch (KS) {
#define KMPAR_FP(V)                                                                              \
  case V:                                                                                        \
    if constexpr (V <= MAXKS)                                                                    \
      return launch_first_one<SPLIT, V, T, true>(X, rsc, n, d, DP, C, rs, D2, A, norms, Apre, s); \
    break;
    KMPAR_FP(1) KMPAR_FP(2) KMPAR_FP(3) KMPAR_FP(4) KMPAR_FP(5) KMPAR_FP(6) KMPAR_FP(7)
    KMPAR_FP(8) KMPAR_FP(9) KMPAR_FP(10) KMPAR_FP(11) KMPAR_FP(12) KMPAR_FP(13) KMPAR_FP(14)
    KMPAR_FP(15) KMPAR_FP(16)
#undef KMPAR_FP
  }
  return hipErrorInvalidValue;
}

hipError_t launch_first_pass(kmpar_dtype dt, int split, int KS, bool prep, const void* X,
                             const float* rsc, int n, int d, int DP, const float* C,
                             const int* rs, float* D2, int* A, float* norms, void* Apre,
                             hipStream_t s) {
  if (prep) {
    if (dt == KMPAR_F32 && split == 3)
      return launch_first_split<3, float>(KS, X, rsc, n, d, DP, C, rs, D2, A, norms, Apre, s);
    if (dt == KMPAR_BF16 && split == 1)
      return launch_first_split<1, bf16_t>(KS, X, rsc, n, d, DP, C, rs, D2, A, norms, Apre, s);
    if (dt == KMPAR_BF16 && split == 2)
      return launch_first_split<2, bf16_t>(KS, X, rsc, n, d, DP, C, rs, D2, A, norms, Apre, s);
    if (dt == KMPAR_FP8_E4M3 && split == 1)
      return launch_first_split<1, fp8_t, 8>(KS, X, rsc, n, d, DP, C, rs, D2, A, norms, Apre, s);
    return hipErrorInvalidValue;
  }
  switch (dt) {
    case KMPAR_F32:
      return launch_first_one<1, 1, float, false>(X, rsc, n, d, DP, C, rs, D2, A, norms, nullptr, s);
    case KMPAR_BF16:
      return launch_first_one<1, 1, bf16_t, false>(X, rsc, n, d, DP, C, rs, D2, A, norms, nullptr, s);
    case KMPAR_FP8_E4M3:
      return launch_first_one<1, 1, fp8_t, false>(X, rsc, n, d, DP, C, rs, D2, A, norms, nullptr, s);
  }
  return hipErrorInvalidValue;
}

// Whether the screen takes its A operands straight from X (no prepared copy):
// BF16 rows (either split: both parts of the K axis are the row itself) or
// FP8 codes read eight at a time when d % 8 == 0, so eight K indices never
// straddle two parts.  FP32 rows use the prepared split terms: building them
// in the screen from 4-byte gathers costs each wave more at its start than
// the prepared copy saves.
bool screen_a_direct(kmpar_dtype dt, int split, int d) {
  if (dt == KMPAR_FP8_E4M3) return split == 1 && d % 8 == 0;  // codes converted in registers
  return dt == KMPAR_BF16 && d % 8 == 0;
}

hipError_t launch_prep_a(kmpar_dtype dt, int split, int KS, const void* X, const float* rsc, int n,
                         int d, float* norms, void* Apre, hipStream_t s) {
  if (dt == KMPAR_F32 && split == 3)
    return launch_prep_a_split<3, float>(KS, X, rsc, n, d, norms, Apre, s);
  if (dt == KMPAR_BF16 && split == 1)
    return launch_prep_a_split<1, bf16_t>(KS, X, rsc, n, d, norms, Apre, s);
  if (dt == KMPAR_BF16 && split == 2)
    return launch_prep_a_split<2, bf16_t>(KS, X, rsc, n, d, norms, Apre, s);
  return hipErrorInvalidValue;
}

hipError_t launch_rownorm(kmpar_dtype dt, const void* X, const float* row_scale, int n, int d,
                          float* norms, hipStream_t s) {
  switch (dt) {
    case KMPAR_F32: return launch_prep_a_one<1, 1, float, false>(X, row_scale, n, d, norms, nullptr, s);
    case KMPAR_BF16: return launch_prep_a_one<1, 1, bf16_t, false>(X, row_scale, n, d, norms, nullptr, s);
    case KMPAR_FP8_E4M3: return launch_prep_a_one<1, 1, fp8_t, false>(X, row_scale, n, d, norms, nullptr, s);
  }
  return hipErrorInvalidValue;
}

template <int SPLIT, bool CODES = false, int MAXKS = kScreenMaxKS>
static hipError_t launch_prep_split(int KS, const float* C, int DP, int d, const int* rs, int m_host,
                                    int max_tiles, float om2g, void* B, float* ncg, const void* X,
                                    const float* rsc, const int* cand, float* scg, int* list_len,
                                    kmpar_stats* st, const int* cperm, hipStream_t s) {
  if (KS < 1 || KS > MAXKS) return hipErrorInvalidValue;
  u16x8* b = static_cast<u16x8*>(B);
  const fp8_t* xc = static_cast<const fp8_t*>(X);
  switch (KS) {
#define KMPAR_PREP(V)                                                                          \
  case V:                                                                                      \
    if constexpr (V <= MAXKS)                                                                  \
      hipLaunchKernelGGL((k_prep_b<SPLIT, V, CODES>), dim3(max_tiles), dim3(64), 0, s, C, DP, d, \
                         rs, m_host, om2g, b, ncg, xc, rsc, cand, scg, list_len, st, cperm);   \
    break;
    KMPAR_PREP(1) KMPAR_PREP(2) KMPAR_PREP(3) KMPAR_PREP(4) KMPAR_PREP(5) KMPAR_PREP(6)
    KMPAR_PREP(7) KMPAR_PREP(8) KMPAR_PREP(9) KMPAR_PREP(10) KMPAR_PREP(11) KMPAR_PREP(12)
    KMPAR_PREP(13) KMPAR_PREP(14) KMPAR_PREP(15) KMPAR_PREP(16)
#undef KMPAR_PREP
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int screen_split(kmpar_dtype dt, bool centers_are_rows) {
  if (dt == KMPAR_F32) return 3;
  // bf16 rows and FP8 codes are exact in bf16; FP32 centers take two terms
  // against bf16 rows (FP8 rows against centers: no screen, direct form)
  if (dt == KMPAR_FP8_E4M3) return centers_are_rows ? 1 : 0;
  return centers_are_rows ? 1 : 2;
}

bool screen_supported(kmpar_dtype dt, bool centers_are_rows, int d) {
  const int sp = screen_split(dt, centers_are_rows);
  return sp != 0 && screen_ksteps(sp, d) <= kScreenMaxKS;
}

// Relative error budget of the screen, as a multiple of S = ||x||^2 + ||c||^2:
// bf16 split truncation (twice the dot), FP32 accumulation of K products,
// FP32 norms, the roundings of the lower-bound arithmetic, the FP32
// direct-form error of the distances it is compared with, and the tile tag
// in the low mantissa bits; times 2 for margin.  FP8 rows add the roundings
// of their decoded elements (fl(s q), twice the dot: 2u S) and of the scaled
// epilogue (s_x s_c, the fma, the bias: 3u, doubled).
float screen_g(kmpar_dtype dt, int split, int d, int tag_bits) {
  const double u = 0x1.0p-24;
  const int K = 32 * screen_ksteps(split, d);
  double split_err = 0.0;
  if (split == 3) split_err = 3.2 * 0x1.0p-16;
  if (split == 2) split_err = 1.1 * 0x1.0p-16;
  // K products plus the -ncg/2 bias, summed in FP32: |sum of terms| <=
  // 1.01 S, doubled by the -2 that turns acc into lb.
  const double acc_err = 2.05 * (K + 1) * u;
  const double misc = (d + 8) * u + 2.0 * (d + 2) * u;
  // |acc| <= |x.c| + ||c||^2 / 2 <= 1.01 S; the tag moves it by less than
  // 2^(TB-23) |acc|, and lb by twice that.
  const double tag_err = 2.02 * std::ldexp(1.0, tag_bits - 23);
  const double scale_err = dt == KMPAR_FP8_E4M3 ? 8.2 * u : 0.0;
  const double safety = 2.0;  // 2G = safety * budget
  return (float)(safety * (split_err + acc_err + misc + tag_err + scale_err) / 2.0);
}

// The candidates of a pass grouped by their norms: a counting sort of the
// candidates into kCandBuckets buckets of log2 ||c||^2 spanning the pass's
// range (every position's order matters only for which tiles can be skipped;
// within a bucket the order is that of the LDS atomics).  cperm[pos] is the
// offset from id0 of the candidate at position pos < m, and tnr[q] an
// interval holding ||c|| of every candidate of tile q (the smallest and
// largest FP64 norm of its 16 rows, rounded to FP32 and widened by 2^-20 on
// each side).  A pass of more than kCandSortMax candidates keeps id order
// and gets intervals [0, inf) (its tiles are never skipped).
__global__ __launch_bounds__(1024) void k_cand_sort(const float* C, int DP, int d, const int* rs,
                                                    int m_host, int* cperm, float2* tnr) {
  __shared__ float key[kCandSortMax];
  __shared__ float skey[kCandSortMax];
  __shared__ int cnt[kCandBuckets];
  __shared__ int sh[1024 / kWave + 1];
  __shared__ float lmin_s[1024 / kWave], lmax_s[1024 / kWave];
  int id0 = 0, m = m_host;
  if (rs) {
    id0 = rs[0];
    m = rs[1] - id0;
  }
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int ntiles = (m + 15) / 16;
  if (m > kCandSortMax) {
    for (int pos = tid; pos < ntiles * 16; pos += 1024) cperm[pos] = pos < m ? pos : -1;
    for (int q = tid; q < ntiles; q += 1024) tnr[q] = make_float2(0.0f, INFINITY);
    return;
  }
  for (int b = tid; b < kCandBuckets; b += 1024) cnt[b] = 0;
  // keys, and the range of log2 of the finite positive ones
  float lo = INFINITY, hi = -INFINITY;
  for (int i = tid; i < m; i += 1024) {
    const float* c = C + (int64_t)(id0 + i) * DP;
    double s2 = 0.0;
    for (int e = 0; e < d; ++e) s2 += (double)c[e] * (double)c[e];
    float k = (float)s2;
    if (!(k <= FLT_MAX)) k = INFINITY;  // NaN goes with the infinite keys
    key[i] = k;
    if (k > 0.0f && k <= FLT_MAX) {
      const float l = log2f(k);
      lo = fminf(lo, l);
      hi = fmaxf(hi, l);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off, kWave));
    hi = fmaxf(hi, __shfl_xor(hi, off, kWave));
  }
  if (lane == 0) {
    lmin_s[wv] = lo;
    lmax_s[wv] = hi;
  }
  __syncthreads();
  lo = INFINITY;
  hi = -INFINITY;
#pragma unroll
  for (int q = 0; q < 1024 / kWave; ++q) {
    lo = fminf(lo, lmin_s[q]);
    hi = fmaxf(hi, lmax_s[q]);
  }
  // bucket 0: zero rows; the last: non-finite; the others split [lo, hi]
  const float scale = hi > lo ? (float)(kCandBuckets - 3) / (hi - lo) : 0.0f;
  auto bucket = [&](float k) {
    if (!(k > 0.0f)) return 0;
    if (!(k <= FLT_MAX)) return kCandBuckets - 1;
    const int b = 1 + (int)((log2f(k) - lo) * scale);
    return b < 1 ? 1 : (b > kCandBuckets - 2 ? kCandBuckets - 2 : b);
  };
  for (int i = tid; i < m; i += 1024) atomicAdd(&cnt[bucket(key[i])], 1);
  __syncthreads();
  // bucket offsets (kCandBuckets == 1024: one bucket per thread)
  int tot;
  const int off = block_excl_scan<int, 1024>(cnt[tid], sh, &tot);
  cnt[tid] = off;  // the scan's barriers order this after every read of cnt
  __syncthreads();
  for (int i = tid; i < m; i += 1024) {
    const float k = key[i];
    const int pos = atomicAdd(&cnt[bucket(k)], 1);
    cperm[pos] = i;
    skey[pos] = k;
  }
  for (int pos = m + tid; pos < ntiles * 16; pos += 1024) cperm[pos] = -1;
  __syncthreads();
  for (int q = tid; q < ntiles; q += 1024) {
    float a2 = INFINITY, b2 = 0.0f;
    for (int pos = q * 16; pos < min(m, q * 16 + 16); ++pos) {
      a2 = fminf(a2, skey[pos]);
      b2 = fmaxf(b2, skey[pos]);
    }
    // keys are rounded to FP32 (relative 2^-24); 2^-20 covers that and sqrt
    tnr[q] = make_float2((float)(sqrt((double)a2) * (1.0 - 0x1.0p-20)),
                         b2 <= FLT_MAX ? (float)(sqrt((double)b2) * (1.0 + 0x1.0p-20)) : INFINITY);
  }
}

hipError_t launch_cand_sort(const float* C, int DP, int d, const int* rs, int m_host, int* cperm,
                            float2* tnr, hipStream_t s) {
  hipLaunchKernelGGL(k_cand_sort, dim3(1), dim3(1024), 0, s, C, DP, d, rs, m_host, cperm, tnr);
  return hipGetLastError();
}

hipError_t launch_prep_b(kmpar_dtype dt, int split, int KS, const float* C, int DP, int d,
                         const int* rs, int m_host, int max_tiles, float om2g, void* B, float* ncg,
                         const void* X, const float* rsc, const int* cand, float* scg,
                         int* list_len, kmpar_stats* st, const int* cperm, hipStream_t s) {
  if (max_tiles <= 0) return hipSuccess;
  const bool fp8 = dt == KMPAR_FP8_E4M3;
  if (fp8 && split == 1) {
    if (!cand || !scg) return hipErrorInvalidValue;
    return launch_prep_split<1, true, 8>(KS, C, DP, d, rs, m_host, max_tiles, om2g, B, ncg, X, rsc,
                                         cand, scg, list_len, st, cperm, s);
  }
  if (fp8) return hipErrorInvalidValue;
  switch (split) {
    case 1: return launch_prep_split<1>(KS, C, DP, d, rs, m_host, max_tiles, om2g, B, ncg, nullptr, nullptr, nullptr, nullptr, list_len, st, cperm, s);
    case 2: return launch_prep_split<2>(KS, C, DP, d, rs, m_host, max_tiles, om2g, B, ncg, nullptr, nullptr, nullptr, nullptr, list_len, st, cperm, s);
    case 3: return launch_prep_split<3>(KS, C, DP, d, rs, m_host, max_tiles, om2g, B, ncg, nullptr, nullptr, nullptr, nullptr, list_len, st, cperm, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_screen(kmpar_dtype dt, int split, int KS, const ScreenArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (dt == KMPAR_F32 && split == 3) return launch_split<3, float>(KS, a, s);
  if (dt == KMPAR_BF16 && split == 1) return launch_split<1, bf16_t>(KS, a, s);
  if (dt == KMPAR_BF16 && split == 2) return launch_split<2, bf16_t>(KS, a, s);
  if (dt == KMPAR_FP8_E4M3 && !a.scg) return hipErrorInvalidValue;
  if (dt == KMPAR_FP8_E4M3 && split == 1) return launch_split<1, fp8_t, 8>(KS, a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_list_reset(int* list_len, kmpar_stats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_list_reset, dim3(1), dim3(64), 0, s, list_len, st);
  return hipGetLastError();
}

}  // namespace kmpar
