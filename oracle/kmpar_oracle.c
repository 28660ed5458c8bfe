/*
 * kmpar_oracle.c -- plain FP64 CPU oracle for k-means|| (Bahmani et al.,
 * "Scalable K-Means++").  TEST INFRASTRUCTURE ONLY: it is called by tests/,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by
 * the library.  It shares no code, header or table with the HIP path.
 *
 * Everything is FP64, loops run in the order the definitions are written
 * (coordinates ascending, candidates ascending, points ascending).  The only
 * parallelism is an OpenMP split of loops whose iterations are independent
 * points; every sum over points is sequential in index order.
 *
 * Parity pins live in tests/test_oracle_*.py.  Functions and what pins them:
 *   orc_philox4x64_10  -- known answers of numpy's independent Philox4x64-10.
 *   orc_nearest        -- scipy cdist('sqeuclidean') brute force.
 *   orc_select         -- exact enumeration / z-tests of the Bernoulli rule.
 *   orc_fold           -- equals orc_nearest against the union of candidates.
 *   orc_weights        -- sums to n; equals a numpy bincount.
 *   orc_kpp_weighted   -- exact enumeration of the pick distribution on tiny
 *                         inputs; w == 1 and C == X gives Algorithm 1.
 *   orc_lloyd_update   -- sklearn's Lloyd iteration (no empty clusters).
 *   orc_exact_keys     -- the law of the smallest key (D^2 sampling) and of the
 *                         l smallest (successive draws without replacement)
 *                         by chi-square against exact enumeration.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Philox4x64-10, from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
 * 64x64->128 multiplies with the round keys bumped by two Weyl constants.
 * ------------------------------------------------------------------------- */
#define PHILOX_M4x64_0 0xD2E7470EE14C6C93ULL
#define PHILOX_M4x64_1 0xCA5A826395121157ULL
#define PHILOX_W64_0 0x9E3779B97F4A7C15ULL
#define PHILOX_W64_1 0xBB67AE8584CAA73BULL

/* Stream tags: one key per independent use of randomness in the method. */
#define ORC_TAG_FIRST 1u /* Algorithm 2 step 1: the uniform first center     */
#define ORC_TAG_ROUND 2u /* Algorithm 2 step 4: per-point Bernoulli draws      */
#define ORC_TAG_RECL 3u  /* step 8: weighted k-means++ picks (Algorithm 1)    */
#define ORC_TAG_EXACT 4u /* D^2 sampling by exponential race: the exact-ell
                            rounds of Section 5.3 and k-means++ on all of X  */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += PHILOX_W64_0;
      k1 += PHILOX_W64_1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M4x64_0 * c0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M4x64_1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Word 0 of the block keyed (seed, tag) at counter (a, b, inst, 0). */
uint64_t orc_word(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t inst) {
  uint64_t ctr[4] = {a, b, inst, 0};
  uint64_t key[2] = {seed, tag};
  uint64_t out[4];
  orc_philox4x64_10(ctr, key, out);
  return out[0];
}

/* Uniform on [0, 1): the top 53 bits of the word, times 2^-53. */
double orc_uniform(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t inst) {
  return (double)(orc_word(seed, tag, a, b, inst) >> 11) * 0x1.0p-53;
}

/* Uniform integer in [0, n): floor(word * n / 2^64), exact in integers. */
int64_t orc_index(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t inst, int64_t n) {
  unsigned __int128 p = (unsigned __int128)orc_word(seed, tag, a, b, inst) * (uint64_t)n;
  return (int64_t)(p >> 64);
}

/* Uniform on (0, 1]: (top 53 bits of the word + 1) * 2^-53, never 0. */
double orc_uniform_open(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t inst) {
  return (double)((orc_word(seed, tag, a, b, inst) >> 11) + 1) * 0x1.0p-53;
}

/* D^2 sampling as an exponential race (Efraimidis & Spirakis, "Weighted
 * random sampling with a reservoir", IPL 2006): point i gets the clock
 * key_i = -ln(V_i) / D2_i, V_i uniform on (0, 1] from tag EXACT at counter
 * (i, t, inst); key_i is exponential with rate D2_i, so the smallest key is
 * point i with probability D2_i / sum_j D2_j (one draw of Algorithm 1's
 * step), and the l smallest keys are l draws without replacement, each in
 * proportion to D^2 among the points not yet drawn.  D2_i = 0 gives +inf:
 * such a point is never drawn. */
void orc_exact_keys(const double* D2, int64_t n, uint64_t seed, int64_t t, uint64_t inst,
                    double* key) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (D2[i] > 0.0)
      key[i] = -log(orc_uniform_open(seed, ORC_TAG_EXACT, (uint64_t)i, (uint64_t)t, inst)) / D2[i];
    else
      key[i] = INFINITY;
  }
}

/* Squared Euclidean distance ||x - c||^2, coordinates in order (Section 3.1). */
static double sqdist(const double* x, const double* c, int32_t d) {
  double s = 0.0;
  for (int32_t j = 0; j < d; ++j) {
    double t = x[j] - c[j];
    s += t * t;
  }
  return s;
}

/* Neumaier-compensated sum of v[0..n) in index order (the cost phi of Section 3.1). */
double orc_sum(const double* v, int64_t n) {
  double s = 0.0, comp = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t = s + v[i];
    if (fabs(s) >= fabs(v[i]))
      comp += (s - t) + v[i];
    else
      comp += (v[i] - t) + s;
    s = t;
  }
  return s + comp;
}

/* Section 3.1: d^2(x, C) = min over centers, and the nearest center (lowest
 * index among equals).  `second` (nullable) receives the second smallest
 * distance, +inf when m == 1. */
void orc_nearest(const double* X, int64_t n, int32_t d, const double* C, int64_t m,
                 int64_t* arg, double* d2, double* second) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double* x = X + i * (int64_t)d;
    double best = INFINITY, snd = INFINITY;
    int64_t bj = -1;
    for (int64_t j = 0; j < m; ++j) {
      double e = sqdist(x, C + j * (int64_t)d, d);
      if (e < best) {
        snd = best;
        best = e;
        bj = j;
      } else if (e < snd) {
        snd = e;
      }
    }
    arg[i] = bj;
    d2[i] = best;
    if (second) second[i] = snd;
  }
}

/* Algorithm 2 step 1: index of the uniformly chosen first center. */
int64_t orc_first_center(int64_t n, uint64_t seed, uint64_t inst) {
  return orc_index(seed, ORC_TAG_FIRST, 0, 0, inst, n);
}

/* Algorithm 2 step 4 for round t (t >= 1): every point is kept
 * independently with probability p = min(1, ell * D2 / phi); the draw for
 * point i in round t is u = U(seed, ROUND, (i, t, inst)) and the point is kept
 * iff u < p.  With phi == 0 nothing is kept.  Writes sel[i] in {0,1} and,
 * when non-null, p[i] and u[i].  Returns the number kept. */
int64_t orc_select(const double* D2, int64_t n, double phi, double ell, uint64_t seed,
                   int64_t t, uint64_t inst, uint8_t* sel, double* p_out, double* u_out) {
  int64_t cnt = 0;
#pragma omp parallel for schedule(static) reduction(+ : cnt)
  for (int64_t i = 0; i < n; ++i) {
    double p = 0.0;
    if (phi > 0.0) {
      p = ell * D2[i] / phi;
      if (p > 1.0) p = 1.0;
    }
    double u = orc_uniform(seed, ORC_TAG_ROUND, (uint64_t)i, (uint64_t)t, inst);
    sel[i] = (u < p) ? 1 : 0;
    cnt += sel[i];
    if (p_out) p_out[i] = p;
    if (u_out) u_out[i] = u;
  }
  return cnt;
}

/* Algorithm 2 step 5 as it acts on d^2(x, C): the m new candidates Cnew get
 * ids first_id, first_id+1, ...; for each point the new candidates are met in
 * id order and the point moves to one only when strictly closer, so among
 * equal distances the lowest id is kept.  S (nullable) tracks the second
 * smallest distance seen. */
void orc_fold(const double* X, int64_t n, int32_t d, const double* Cnew, int64_t m,
              int64_t first_id, double* D2, int64_t* A, double* S) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double* x = X + i * (int64_t)d;
    for (int64_t j = 0; j < m; ++j) {
      double e = sqdist(x, Cnew + j * (int64_t)d, d);
      if (e < D2[i]) {
        if (S) S[i] = D2[i];
        D2[i] = e;
        A[i] = first_id + j;
      } else if (S && e < S[i]) {
        S[i] = e;
      }
    }
  }
}

/* Algorithm 2 step 7: w_c = number of points whose nearest candidate is c. */
void orc_weights(const int64_t* A, int64_t n, int64_t ncand, int64_t* w) {
  memset(w, 0, sizeof(int64_t) * (size_t)ncand);
  for (int64_t i = 0; i < n; ++i) w[A[i]] += 1;
}

/* Inclusive running sums P_j = sum_{i<=j} v_i in index order; returns the
 * smallest j with P_j > thr, or the largest j with v_j > 0 when rounding left
 * thr at or above the total (or -1 if every v_j is 0). */
static int64_t inverse_cdf(const double* v, int64_t m, double thr, double* P) {
  double run = 0.0;
  int64_t last_pos = -1, pick = -1;
  for (int64_t j = 0; j < m; ++j) {
    run += v[j];
    P[j] = run;
    if (v[j] > 0.0) last_pos = j;
    if (pick < 0 && run > thr) pick = j;
  }
  return pick >= 0 ? pick : last_pos;
}

/* Algorithm 2 step 8 with k-means++ (Algorithm 1) on the weighted candidates,
 * the reclustering the experiments use: the first pick has probability
 * w_j / sum(w); pick s >= 1 has probability w_j E_j / T with
 * E_j = min over earlier picks of ||c_j - c_pick||^2 and T = sum_j w_j E_j.
 * Pick s uses u = U(seed, RECL, (s, 0, inst)) and takes the smallest j with
 * P_j > u * T.
 *
 * `follow` (nullable) holds another implementation's picks: where they differ
 * from this oracle's pick, the other pick is accepted (and counted in
 * *n_flag) if u*T lies within tol*T of an interval boundary that makes it the
 * pick, else counted in *n_bad; the followed pick is kept either way so the
 * comparison can go on.  Returns the number of picks made (< k when every
 * remaining candidate has zero weighted distance). */
int64_t orc_kpp_weighted(const double* C, int64_t m, int32_t d, const double* w, int64_t k,
                         uint64_t seed, uint64_t inst, const int64_t* follow, double tol,
                         int64_t* picks, int64_t* n_flag, int64_t* n_bad) {
  double* E = (double*)malloc(sizeof(double) * (size_t)m);
  double* v = (double*)malloc(sizeof(double) * (size_t)m);
  double* P = (double*)malloc(sizeof(double) * (size_t)m);
  int64_t made = 0;
  if (n_flag) *n_flag = 0;
  if (n_bad) *n_bad = 0;
  for (int64_t j = 0; j < m; ++j) E[j] = 1.0; /* step 0: weights alone */
  for (int64_t s = 0; s < k; ++s) {
    for (int64_t j = 0; j < m; ++j) v[j] = w[j] * E[j];
    double T = 0.0;
    for (int64_t j = 0; j < m; ++j) T += v[j];
    if (!(T > 0.0)) break;
    double u = orc_uniform(seed, ORC_TAG_RECL, (uint64_t)s, 0, inst);
    double thr = u * T;
    int64_t pick = inverse_cdf(v, m, thr, P);
    if (follow && follow[s] != pick) {
      int64_t g = follow[s];
      int ok = 0;
      if (g >= 0 && g < m && v[g] > 0.0) {
        double lo = (g > 0) ? P[g - 1] : 0.0, hi = P[g];
        ok = (hi > thr - tol * T) && (lo <= thr + tol * T);
      }
      if (ok) {
        if (n_flag) *n_flag += 1;
      } else {
        if (n_bad) *n_bad += 1;
      }
      pick = (g >= 0 && g < m) ? g : pick;
    }
    picks[s] = pick;
    made = s + 1;
    const double* cp = C + pick * (int64_t)d;
    for (int64_t j = 0; j < m; ++j) {
      double e = sqdist(C + j * (int64_t)d, cp, d);
      if (s == 0 || e < E[j]) E[j] = e;
    }
  }
  free(E);
  free(v);
  free(P);
  return made;
}

/* One Lloyd update (Section 1, Section 3.1): each center moves to the
 * centroid of the points assigned to it; a center with no points stays.
 * Sums run over points in index order.  counts (nullable) receives the
 * cluster sizes. */
void orc_lloyd_update(const double* X, int64_t n, int32_t d, const int64_t* a, int64_t k,
                      double* C, int64_t* counts) {
  double* sum = (double*)calloc((size_t)k * (size_t)d, sizeof(double));
  int64_t* cnt = (int64_t*)calloc((size_t)k, sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = a[i];
    cnt[c] += 1;
    for (int32_t j = 0; j < d; ++j) sum[c * d + j] += X[i * (int64_t)d + j];
  }
  for (int64_t c = 0; c < k; ++c) {
    if (cnt[c] > 0)
      for (int32_t j = 0; j < d; ++j) C[c * d + j] = sum[c * d + j] / (double)cnt[c];
    if (counts) counts[c] = cnt[c];
  }
  free(sum);
  free(cnt);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
