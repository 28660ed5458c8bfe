// Host-side launchers of the kmpar kernels (internal to libkmpar.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <map>

#include "../../include/kmpar.h"
#include "geometry.hpp"

namespace kmpar {

inline int padded_dim(int d) { return padded_dim_hd(d); }

// Parameters of one distance-fold pass: every listed point meets the m
// candidate rows C[id0 .. id0+m) (DP-padded FP32) and keeps the nearest.
struct FoldArgs {
  const void* X;
  const float* row_scale;
  int n;
  int d;
  const float* C;        // candidate rows, row r at C + r*DP
  const int* rs;         // device: id0 = rs[0], m = rs[1] - rs[0]  (nullable)
  int m_host;            // used when rs == nullptr
  int id0_host;
  float* D2;
  int* A;
  int first;             // 1: previous D2/A are ignored
  const int* list;       // nullable: only points list[0 .. *list_len)
  const int* list_len;
  int list_cap;          // upper bound of *list_len
  float* norms;          // nullable: also write ||x||^2 (FP32) of every point
  int4* rpart;           // nullable: kRescanMaxItems * kRescanPts slice winners of a split rescan
                         // (distance bits, id, second distance bits, unused)
  float* S;              // nullable: each point's second-smallest distance, kept with D2 / A
  // Candidate-sharded fold (nullable): the m candidates are cut into
  // `shards` consecutive slices, block row blockIdx.y takes slice
  // blockIdx.y, and each point's (distance, id) minimum over the slice is
  // merged into packed[i] = (FP32 bits of the distance) << 32 | id with an
  // integer atomic minimum instead of being written to D2 / A.
  unsigned long long* packed;
  int shards;
};

hipError_t launch_fold_direct(kmpar_dtype dt, int DP, const FoldArgs& a, hipStream_t s);
// packed[i] -> A[i] (the id) and, when D2 != nullptr, D2[i] (the distance).
hipError_t launch_unpack_min(const unsigned long long* packed, int n, int* A, float* D2,
                             hipStream_t s);
// Listed points only (a.list, a.list_len, a.list_cap), one wave per point.
hipError_t launch_rescan(kmpar_dtype dt, int DP, const FoldArgs& a, hipStream_t s);

// REFINED screen (see screen_mfma.hip).
struct ScreenArgs {
  const void* X;
  const float* row_scale;
  int n;
  int d;
  int DP;
  const float* C;        // FP32 candidate rows (DP-padded) used for refinement
  const int* rs;         // device: id0 = rs[0], m = rs[1] - rs[0]  (nullable)
  int m_host;
  int id0_host;
  const void* Apre;      // bf16 A operands from launch_prep_a (nullptr: read X directly)
  const void* B;         // bf16 B operands from launch_prep_b
  const float* ncg;      // (1 - 2G) ||c||^2 per candidate, +inf past m
  const float* scg;      // FP8 rows: each candidate's scale (0 for a trivial bound);
                         // nullptr otherwise
  const float* norms;    // ||x||^2 per point
  float oneminus2g;
  float* D2;
  int* A;
  float* S;              // nullable: second-smallest distance per point (see screen_body)
  int first;
  int* list;             // points the screen could not settle
  int* list_len;
  kmpar_stats* stats;    // nullable: receives the listed counts
  int tag_bits;          // > 0: single-group screen, tiles tagged by their index in the pass
  const int* cperm;      // nullable: candidate (offset from id0) at each tile position
  const float2* tnr;     // nullable: ||c|| interval of each tile (with cperm)
};

int screen_split(kmpar_dtype dt, bool centers_are_rows);
bool screen_supported(kmpar_dtype dt, bool centers_are_rows, int d);
// Error constant G of the screen's lower bound with tag_bits bits of tag.
float screen_g(kmpar_dtype dt, int split, int d, int tag_bits);
// B operands of the candidates C[rs[0] ..) (or C[0 .. m_host)), their biases
// and, for FP8 rows, their scales: FP8 rows (split 1, against rows of X)
// take the candidates' e4m3 codes from X rows cand[id].  It also adds the
// previous pass's *list_len to st->n_rescanned (st nullable) and clears it.
hipError_t launch_prep_b(kmpar_dtype dt, int split, int KS, const float* C, int DP, int d,
                         const int* rs, int m_host, int max_tiles, float om2g, void* B, float* ncg,
                         const void* X, const float* rsc, const int* cand, float* scg,
                         int* list_len, kmpar_stats* st, const int* cperm, hipStream_t s);
// The pass's candidates in norm order (cperm) and the norm interval of each
// tile of 16 (tnr), for the screen.
hipError_t launch_cand_sort(const float* C, int DP, int d, const int* rs, int m_host, int* cperm,
                            float2* tnr, hipStream_t s);
hipError_t launch_screen(kmpar_dtype dt, int split, int KS, const ScreenArgs& a, hipStream_t s);
bool screen_a_direct(kmpar_dtype dt, int split, int d);
// The screen's A operands and, when norms != nullptr, ||x||^2, from one read of X.
hipError_t launch_prep_a(kmpar_dtype dt, int split, int KS, const void* X, const float* rsc, int n,
                         int d, float* norms, void* Apre, hipStream_t s);
hipError_t launch_list_reset(int* list_len, kmpar_stats* st, hipStream_t s);
// The first pass against candidate rs[0] (D2, A, optional norms), fused with
// the A operands of the screen when prep.
hipError_t launch_first_pass(kmpar_dtype dt, int split, int KS, bool prep, const void* X,
                             const float* rsc, int n, int d, int DP, const float* C,
                             const int* rs, float* D2, int* A, float* norms, void* Apre,
                             hipStream_t s);
// ||x||^2 in FP32, coordinates in ascending order (the first pass's arithmetic).
hipError_t launch_rownorm(kmpar_dtype dt, const void* X, const float* row_scale, int n, int d,
                          float* norms, hipStream_t s);

hipError_t launch_first(int n, uint64_t seed, uint64_t inst, int* cand_point, int* rs,
                        kmpar_stats* st, hipStream_t s);
hipError_t launch_gather(kmpar_dtype dt, const void* X, const float* row_scale, int d, int DP,
                         const int* cand_point, const int* rs, int t, int cap_round, float* Call,
                         float* CallT, int ldT, hipStream_t s);
hipError_t launch_phi(const float* D2, int n, double* part, double* out, hipStream_t s);
// Round t's Bernoulli draws (Algorithm 2 step 4) and their ordered
// compaction; draws within `band` (relative to p) are counted in
// st->flagged_draws.
hipError_t launch_draw(const float* D2, int n, const double* phi, double ell, uint64_t seed, int t,
                       uint64_t inst, double band, int* cnt, uint64_t* keep, int* scan_total,
                       int* rs, int cap_round, int* cand_point, kmpar_stats* st, hipStream_t s);
// The ordered compaction of round t from per-block kept counts cnt[] and
// keep masks (one bit per point, kDrawChunk points per block): exclusive
// scan of the counts, commit of the round (rs[t+1] = rs[t] + m_t, capped at
// cap_round, stats), then the kept point indices in increasing order.
hipError_t launch_round_compact(int n, int* cnt, const uint64_t* keep, int* scan_total, int* rs,
                                int t, int cap_round, int* cand_point, kmpar_stats* st,
                                hipStream_t s);
// Relative error band of an FP32 direct-form squared distance over d
// coordinates, doubled: 2 (d + 2) 2^-24.
__host__ __device__ inline double fp32_flag_band(int d) { return 2.0 * (d + 2) * 0x1.0p-24; }
// Whether a recluster pick could have fallen into the neighbouring interval:
// every mass w_j E_j carries the relative error of its FP32 distance, at most
// band / 2, so a running sum P and the threshold u T move by at most band / 2
// times themselves, and their difference by (band / 2)(P + u T) (the FP64
// roundings add a relative 2^-50 margin).  [lo, hi) is the picked interval.
__host__ __device__ inline bool pick_near_end(double thr, double lo, double hi, double band) {
  const double b = 0.5 * band + 0x1.0p-50;
  return thr - lo <= b * (thr + lo) || hi - thr <= b * (hi + thr);
}
hipError_t launch_finish_rounds(const int* rs, int rounds, kmpar_stats* st, hipStream_t s);
// st->flagged_argmins += #{i : S[i] <= (1 + band) D2[i]}.
hipError_t launch_flag_argmins(const float* D2, const float* S, int n, double band,
                               kmpar_stats* st, hipStream_t s);
hipError_t launch_fill_i32(int* p, int v, int64_t count, hipStream_t s);
// Step-7 weights w[0 .. nbins) of the assignment A (an LDS histogram per
// block while nbins fits a CU's LDS, else global atomics).
hipError_t launch_hist(const int* A, int n, int* w, int nbins, int num_cu, hipStream_t s);
// Step-8 recluster in one workgroup when E and the nearest-pick ids fit LDS.
constexpr size_t kReclBlockLdsMax = 140 * 1024;
size_t recluster_block_lds(int capT, int k);
hipError_t launch_recluster_block(const float* CallT, int capT, int d, const int* w,
                                  const int* rs_end, int k, uint64_t seed, uint64_t inst,
                                  int* picks, float* centers, kmpar_stats* st, double band,
                                  hipStream_t s);
// Step-8 recluster over G workgroups (see aux_kernels.hip).
// Grid of the multi-workgroup recluster for up to capT candidates of DP
// floats on num_cu CUs: G blocks of at most `fit` candidates each, rows in
// LDS or (lds_rows false, or forced by global_rows) in global memory, `lds`
// dynamic LDS bytes per block.  False when even global rows do not fit.
struct ReclPlan {
  int G;
  int fit;
  bool lds_rows;
  size_t lds;
  int num_cu;  // CUs of the device the plan is for
};
constexpr int kXcds = 8;  // XCDs of the chip, each with its own L2
constexpr int kReclMaxBlocks = 512;
bool recluster_plan(int capT, int DP, int num_cu, bool global_rows, ReclPlan* p);
hipError_t launch_recluster(const float* Call, int DP, int d, const int* w, const int* rs_end,
                            int k, uint64_t seed, uint64_t inst, const ReclPlan& plan,
                            double* udraw, double* part, float* prow, int* picks,
                            float* centers, kmpar_stats* st, double band, hipStream_t s);
hipError_t launch_pad_rows(const float* C, int m, int d, int DP, float* Cpad, hipStream_t s);
hipError_t launch_copy_i32(const int* src, int* dst, int64_t count, hipStream_t s);

// Lloyd centroid update by a deterministic counting sort.
struct LloydWs {
  int* bcnt;      // (k + 1) * nbs: clusters 0 .. k-1, then points with no valid center
  int* scan_tmp;  // ceil((k + 1) * nbs / kScanTile) + 1
  int* sorted;    // n
  int* cstart;    // k + 1
  int* coff;      // k + 1
  double* part;   // (ceil(n / kSegChunk) + k) * d
};
hipError_t launch_lloyd_update(kmpar_dtype dt, const void* X, const float* row_scale, int n, int d,
                               const int* A, int k, float* C, const LloydWs& w, hipStream_t s);

// Exact-ell rounds and k-means++ by an exponential race (exact.hip).
// State of one round's radix select of the ell-th smallest key.
struct ExactState {
  unsigned long long prefix;  // the key bits fixed so far (after the last level: tau)
  int need;                   // 1-based rank of the wanted key within the current bucket
  int m;                      // points the round takes: min(ell, points with D^2 > 0)
  int tie_need;               // keys equal to tau that are taken
  int tie_count;              // keys equal to tau
  int tie_last;               // index of the last key equal to tau taken (INT_MAX: all)
  int pad;
};
struct ExactWs {
  unsigned long long* keys;  // [n] key bits of the round
  int* hist;                 // [exact_hist_bins()] zero between rounds
  ExactState* state;
};
size_t exact_keys_bytes(int64_t n);
int exact_hist_bins();
// Round t of the exact-ell variant (Section 5.3): the min(ell, #{D^2 > 0})
// points with the smallest race keys, appended in index order (counts, masks
// and compaction as launch_draw); keys within `band` of tau are counted in
// st->flagged_draws.
hipError_t launch_exact_round(const float* D2, int n, int ell, uint64_t seed, int t, uint64_t inst,
                              double band, const ExactWs& w, int* cnt, uint64_t* keep,
                              int* scan_total, int* rs, int cap_round, int* cand_point,
                              kmpar_stats* st, hipStream_t s);
struct KppWs {
  float* D2;                // [n]
  unsigned long long* pkey; // [ceil(n / 64)] per-block smallest key
  int* pidx;                // [ceil(n / 64)] its point
  double* pphi;             // [ceil(n / 64)] per-block FP64 sum of D^2
  float* crow;              // [d] the latest center
  int* stop;                // 1 once every point lies on a center
  unsigned long long* qkey; // [kKppQ] the same over runs of block partials
  int* qidx;                // [kKppQ]
  double* qphi;             // [kKppQ]
};
// k-means++ on all of X (Algorithm 1) with race-key draws: k - 1 steps of
// one fold + key pass over X and one pick.
hipError_t launch_kmeanspp(kmpar_dtype dt, const void* X, const float* rsc, int n, int d, int k,
                           uint64_t seed, uint64_t inst, const KppWs& w, int* picks,
                           float* centers, double* phi_steps, kmpar_stats* st, hipStream_t s);
// *out = number of i < n with a[i] != b[i].
hipError_t launch_count_changed(const int* a, const int* b, int n, int* out, hipStream_t s);

// Batched k-means|| (batched.hip).
constexpr int kBatchMaxGroups = 24;
size_t batched_workspace(const kmpar_instance* inst, int count, int rounds, int* G_out, int* dps);
// Tile shapes of the batched distance pass (candidates per step) chosen by
// timing on the first batch of each (dtype, padded row length).
struct BatchTuner {
  bool enabled = true;
  std::map<int, int> cb;  // key(dtype, DP) -> candidates per step
  static int key(int dt, int DP) { return dt * 4096 + DP; }
};
// Runs one launch, bracketed by the caller's timing when it profiles.
using LaunchTimer = std::function<hipError_t(const std::function<hipError_t()>&)>;
// fold_timer (nullable) brackets every grouped fold launch except the
// tuner's trial launches.
hipError_t launch_batched(kmpar_dtype dt, const kmpar_instance* ih, const kmpar_instance* idev,
                          int count, int rounds, uint64_t seed, void* ws, const kmpar_trace* tr,
                          BatchTuner* tuner, const LaunchTimer* fold_timer, hipStream_t s);

}  // namespace kmpar
