/*
 * kmpar.h -- C ABI of libkmpar.so: k-means|| (Bahmani, Moseley, Vattani,
 * Kumar, Vassilvitskii, "Scalable K-Means++", PVLDB 2012) on AMD MI355X.
 *
 * Problem statement (Section 3.1): X = {x_1..x_n} in R^d, an integer k; the
 * cost of a center set C is phi_X(C) = sum_x min_{c in C} ||x - c||^2; every
 * center defines the cluster of points closer to it than to any other.
 *
 * Conventions shared by every call
 *  - X is row-major n x d.  dtype KMPAR_F32: float; KMPAR_BF16: bfloat16 bits
 *    (uint16); KMPAR_FP8_E4M3: OCP e4m3 bytes with one float scale per row
 *    (x_ij = decode(q_ij) * row_scale[i]).  row_scale must be NULL for the
 *    other dtypes.
 *  - Every array argument is a DEVICE pointer owned by the caller and at least
 *    16-byte aligned.  The library never allocates device memory: scratch
 *    comes from the caller's workspace `ws` of `ws_bytes` bytes, sized with
 *    kmpar_workspace_size().  Its contents on entry do not matter.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls only enqueue
 *    work: outputs are valid once the stream has been synchronised.  Calls
 *    make no host synchronisation and may be captured in a hipGraph.
 *  - Arguments are validated on the host before any HIP call.  Return value
 *    0 (KMPAR_OK) or a negative kmpar_status; kmpar_last_error() gives text.
 *  - Limits: 1 <= n < 2^31, 1 <= d <= 256, 1 <= k <= n, k <= 16384,
 *    rounds <= KMPAR_MAX_ROUNDS.
 *  - Results are deterministic: the same inputs, seed, mode and device give
 *    bit-identical outputs (every reduction runs in a fixed order).
 *  - Calls that share one workspace or one context must not overlap.  Calls
 *    with their own context and workspace may run concurrently on different
 *    streams of one device, and give the results they give alone.  Step 8 of
 *    kmpar_init runs on a few workgroups that wait for one another; a
 *    concurrent kernel that holds the compute units can delay them, and a
 *    wait that exceeds its bound (seconds) ends the call with status
 *    KMPAR_E_HIP in kmpar_stats rather than hanging.
 */
#ifndef KMPAR_H_
#define KMPAR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KMPAR_MAX_ROUNDS 64

typedef enum kmpar_dtype { KMPAR_F32 = 0, KMPAR_BF16 = 1, KMPAR_FP8_E4M3 = 2 } kmpar_dtype;

/* PLAIN_FP32: every point-center distance in FP32 direct form
 * sum_j (x_j - c_j)^2.  REFINED: distances screened on the matrix cores
 * from ||x||^2 - 2 x.c + ||c||^2 with a rigorous error band (bf16 operands:
 * BF16 rows and the codes of FP8 rows as they are, FP32 values split into
 * two or three bf16 terms; FP8 row scales applied after the products), and
 * every decision the band cannot settle recomputed in FP32 direct form, so
 * both modes return the same results bit for bit.  FP8 rows are screened in
 * kmpar_init; their assignment passes (kmpar_assign, kmpar_cost,
 * lloyd_step, kmpar_lloyd) use the direct form in both modes. */
typedef enum kmpar_mode { KMPAR_MODE_PLAIN_FP32 = 0, KMPAR_MODE_REFINED = 1 } kmpar_mode;

typedef enum kmpar_status {
  KMPAR_OK = 0,
  KMPAR_E_INVAL = -1,     /* argument out of range, NULL or misaligned pointer */
  KMPAR_E_WORKSPACE = -2, /* ws_bytes smaller than kmpar_workspace_size()      */
  KMPAR_E_HIP = -3,       /* a HIP call failed; text in kmpar_last_error()     */
  KMPAR_E_TOOFEW = -4,    /* (stats.status) fewer than k distinct candidates  */
  KMPAR_E_OVERFLOW = -5,  /* (stats.status) a round kept more points than the
                             per-round capacity; that round was truncated     */
  KMPAR_E_NODEVICE = -6   /* context created without a device                 */
} kmpar_status;

/* Which call a workspace is sized for. */
typedef enum kmpar_op {
  KMPAR_OP_INIT = 0,
  KMPAR_OP_COST = 1,
  KMPAR_OP_ASSIGN = 2,
  KMPAR_OP_LLOYD = 3,    /* lloyd_step, kmpar_lloyd, kmpar_lloyd_until_stable */
  KMPAR_OP_KMEANSPP = 4, /* kmpar_kmeanspp                                   */
  KMPAR_OP_ASSIGN_SHARDED = 5 /* kmpar_assign_sharded (k = m, up to 2^24)     */
} kmpar_op;

typedef struct kmpar_ctx kmpar_ctx;

/* Per-call record of kmpar_init, written on the device (caller-owned device
 * memory of kmpar_sizeof_stats() bytes). */
typedef struct kmpar_stats {
  double phi[KMPAR_MAX_ROUNDS + 1];          /* phi_X(C): [0] = psi after the first
                                                center (Alg. 2 step 2), [t] after
                                                round t (steps 4-5)               */
  int32_t round_count[KMPAR_MAX_ROUNDS + 1]; /* |C'_t| kept in round t; [0] = 1   */
  int32_t n_candidates;                      /* |C| after the last round          */
  int32_t n_centers;                         /* centers written (k unless TOOFEW) */
  int32_t status;                            /* KMPAR_OK, _E_TOOFEW or _E_OVERFLOW */
  int32_t n_rescanned;                       /* REFINED: point passes the screen
                                                could not settle (recomputed in
                                                direct form), summed over passes  */
  /* Decisions taken inside the FP32 error band, band = 2 (d + 2) 2^-24 (the
   * relative error bound of an FP32 direct-form squared distance, doubled):
   * they may legitimately differ from exact arithmetic and are counted, not
   * hidden (the replay of an FP64 reference accepts exactly these). */
  int32_t flagged_draws;                     /* round draws with |u - p| <= band p,
                                                summed over rounds (step 4)       */
  int32_t flagged_picks;                     /* recluster picks whose u T lies
                                                within (band / 2)(P + u T) of an
                                                end P of the picked interval: the
                                                masses' FP32 distances could have
                                                moved it across (step 8)          */
  int32_t flagged_argmins;                   /* kmpar_init: points whose second-
                                                nearest candidate lies within
                                                (1 + band) D^2 of the nearest
                                                (step 7; 0 in batched calls)     */
  int32_t reserved;
} kmpar_stats;

/* Optional device outputs of kmpar_init for inspection (each may be NULL). */
typedef struct kmpar_trace {
  int32_t* cand_point;  /* [max_candidates] point index of candidate id c; ids are
                           given in append order: round, then point index      */
  int32_t* cand_weight; /* [max_candidates] Step-7 weight w_c                    */
  int32_t* center_cand; /* [k] candidate id of the s-th recluster pick            */
  int32_t* assign;      /* [n] id of the nearest candidate after the last round   */
  float* d2;            /* [n] D^2(x, C) after the last round (FP32)             */
} kmpar_trace;

/* Tuning options of a context. */
typedef enum kmpar_option {
  /* Step-8 recluster of kmpar_init: 0 = automatic (2 when the CUs' LDS can
   * hold every candidate row, else 3), 1 = one workgroup (candidate E values
   * in LDS, rows streamed), 2 = several workgroups with LDS-resident row
   * slices, 3 = several workgroups reading the rows from global memory.
   * All give the same picks up to FP64 summation order. */
  KMPAR_OPT_RECLUSTER_PATH = 0,
  /* Tile shapes of kmpar_init_batched's distance pass: 1 (default) = the
   * first batch that meets a (dtype, padded row length) times every
   * candidates-per-step variant of that group's fold on its first round
   * (re-applying a fold changes nothing, so results do not depend on it) and
   * the context keeps the fastest for later batches; 0 = fixed defaults.
   * Tuning synchronises the stream once per new shape and is skipped while
   * the stream is being captured into a graph. */
  KMPAR_OPT_BATCH_AUTOTUNE = 1,
  /* Round draws of kmpar_init: 0 (default) = Algorithm 2, every point kept
   * independently with probability min(1, ell d^2(x) / phi); 1 = the
   * exact-ell variant of Section 5.3, exactly min(ell, #{d^2 > 0}) points
   * per round, drawn in proportion to d^2 without replacement (ell must then
   * be an integer).  Those draws are an exponential race: point i gets the
   * key -ln(V) / d^2(x_i) with V = ((w >> 11) + 1) 2^-53, w from Philox tag 4
   * at counter (i, t, 0), and the ell smallest keys are kept (ties: lower
   * index); with ell = 1 and rounds = k - 1 the candidates are exactly the
   * picks of kmpar_kmeanspp with the same seed.  stats->flagged_draws then
   * counts keys within the FP32 band of the round's threshold key. */
  KMPAR_OPT_SAMPLING = 2
} kmpar_option;
int kmpar_set_option(kmpar_ctx* ctx, kmpar_option opt, int64_t value);

/* The batched tile shapes tuned so far, one entry per (dtype, padded row
 * length): up to `cap` entries are written to dtype[], dp[] (padded row
 * length) and cb[] (the fold variant: 1, 2, 4 or 8 candidates per step, or
 * 200 for rows of 65 to 128 elements split over two waves); *count receives
 * the number of entries.  Host memory; no device work. */
int kmpar_batch_tiles(const kmpar_ctx* ctx, int32_t* dtype, int32_t* dp, int32_t* cb, int32_t cap,
                      int32_t* count);

/* Kernel timing for measurement: while enabled, every launch of a distance
 * kernel (the fold of Algorithm 2 steps 4-5 and of the assignment passes) is
 * bracketed by two hipEvents recorded on the call's stream.
 * kmpar_profile_read() synchronises on those events and reports, for kernel
 * slot `slot` (0 = direct-form fold, 1 = REFINED screen, 2 = rescan of the
 * points the screen listed, 3 = the grouped folds of kmpar_init_batched),
 * the number of launches, their summed duration in milliseconds and their
 * summed algorithmic work in point-center pairs (n * m per launch, m read
 * back from the device after the call; 0 for slot 3, whose launches cover
 * many instances: the caller sums n_i |C_i| from the stats); reading also
 * clears the slot.  Disabled by default; enabling adds one
 * event pair per launch and must not be used under graph capture. */
int kmpar_profile_enable(kmpar_ctx* ctx, int on);
int kmpar_profile_read(kmpar_ctx* ctx, int slot, int64_t* launches, double* total_ms,
                       double* pairs);

/* Creates a context bound to HIP device `hip_device`, or a host-only context
 * when hip_device == -1 (validation and size queries only; compute calls then
 * return KMPAR_E_NODEVICE).  Returns KMPAR_E_HIP when the device cannot be
 * queried. */
int kmpar_create(int hip_device, kmpar_mode mode, kmpar_ctx** out);
void kmpar_destroy(kmpar_ctx* ctx);
const char* kmpar_strerror(int status);
const char* kmpar_last_error(const kmpar_ctx* ctx);
size_t kmpar_sizeof_stats(void);

/* Upper bound on |C| that kmpar_init keeps: 1 + rounds * per-round capacity,
 * where the capacity min(n, L + 12 isqrt(L) + 76), L = ceil(ell), is at
 * least ell + 12 sqrt(ell) + 64: more than 12 standard deviations above the
 * expected ell points per round (Section 3.3: each round keeps ell points in
 * expectation). */
int kmpar_max_candidates(int64_t n, double ell, int32_t rounds, int64_t* out);

/* Workspace bytes for `op` at the given sizes (k = number of centers m for
 * COST/ASSIGN/LLOYD; ell and rounds are ignored there).  Host only. */
int kmpar_workspace_size(const kmpar_ctx* ctx, kmpar_op op, int64_t n, int32_t d, int32_t k,
                         double ell, int32_t rounds, kmpar_dtype dtype, size_t* bytes_out);

/* Algorithm 2 (Section 3.3), k-means|| initialisation:
 *  1. the first center is a uniformly random point;
 *  2. psi = phi_X(C);
 *  3-6. for `rounds` rounds each point x is kept independently with
 *     probability min(1, ell * d^2(x, C) / phi_X(C)) and the kept points join C;
 *  7. w_c = number of points whose nearest candidate is c (ties: lowest id);
 *  8. the weighted candidates are reclustered into k centers with k-means++
 *     (Algorithm 1, weights multiplying the D^2 probabilities), as in the
 *     experiments (Section 4.2).
 * Randomness: Philox4x64-10 keyed (seed, tag) at counter (a, b, inst, 0):
 * tag 1 first center (a=b=0), tag 2 round draws (a = point index, b = round
 * t >= 1), tag 3 recluster picks (a = pick number s, b = 0); inst = 0.
 * Output: `centers` [k x d] FP32 in pick order (each is a row of X).  `stats`
 * (device, nullable) and `trace` (host struct of device pointers, nullable).
 * Errors found on the device (too few candidates, capacity overflow) are
 * reported in stats->status. */
int kmpar_init(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
               int64_t n, int32_t d, int32_t k, double ell, int32_t rounds, uint64_t seed,
               float* centers, void* ws, size_t ws_bytes, kmpar_stats* stats,
               const kmpar_trace* trace, void* stream);

/* phi_X(C) (Section 3.1) of the m centers C [m x d FP32] into *phi (device
 * double), summed in FP64 in a fixed order. */
int kmpar_cost(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
               int64_t n, int32_t d, const float* C, int32_t m, double* phi, void* ws,
               size_t ws_bytes, void* stream);

/* Size of the fixed device scratch that kmpar_cost_noalloc works in. */
#define KMPAR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* kmpar_cost without a workspace, for callers that cannot allocate device
 * memory (code under hipGraph capture that may not call hipMalloc, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, same
 * launches and bit-identical result as kmpar_cost, but its scratch is a
 * fixed KMPAR_NOALLOC_SCRATCH_BYTES (64 MiB) array that the library holds on
 * every GPU it runs on until the process ends; nothing is allocated or
 * freed, and no event is created (profiling is skipped for this call).
 * Returns KMPAR_E_WORKSPACE, before any HIP call, when the call needs more
 * scratch than that: kmpar_workspace_size(ctx, KMPAR_OP_COST, ...) must not
 * exceed it (about 8 n + 4 m d bytes for a PLAIN_FP32 context, n up to
 * about eight million; REFINED contexts also need the screen's operands,
 * up to 272 bytes per point).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other contexts,
 * other threads) race and must be serialised by the caller. */
int kmpar_cost_noalloc(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                       int64_t n, int32_t d, const float* C, int32_t m, double* phi,
                       void* stream);

/* Nearest center of every point (Section 3.1; ties to the lowest index):
 * assign [n] int32, d2 [n] FP32 squared distance (nullable). */
int kmpar_assign(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                 int64_t n, int32_t d, const float* C, int32_t m, int32_t* assign, float* d2,
                 void* ws, size_t ws_bytes, void* stream);

/* The nearest of m centers for every point when the center set is large
 * (Section 3.5, last paragraph: each mapper holds a slice C' of the centers
 * and emits <x; argmin over C'>, and the reducer takes the minimum): the m
 * centers [m x d FP32] are cut into `shards` consecutive slices, every
 * slice is folded over all points concurrently in FP32 direct form, and
 * each point's (distance, id) minimum over a slice is merged into one
 * packed 64-bit word per point (distance bits, then id) with an integer
 * atomic minimum, which keeps the smallest distance and, among equal ones,
 * the lowest id -- the result of kmpar_assign bit for bit, for m up to
 * 2^24 (kmpar_assign takes up to 16384).  1 <= shards <= min(m, 256); more
 * shards put more workgroups on few points.  Outputs: assign [n], d2 [n]
 * (nullable), phi (device double, nullable) = the cost, summed in FP64 in a
 * fixed order.  Workspace: kmpar_workspace_size(KMPAR_OP_ASSIGN_SHARDED,
 * n, d, m, ...). */
int kmpar_assign_sharded(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                         int64_t n, int32_t d, const float* C, int32_t m, int32_t shards,
                         int32_t* assign, float* d2, double* phi, void* ws, size_t ws_bytes,
                         void* stream);

/* One Lloyd iteration (Section 1; Section 3.1): assign every point to its
 * nearest center, then replace each center by the centroid of its points; a
 * center with no points is kept.  C [k x d FP32] is updated in place.
 * assign [n] (nullable) receives the assignment to the INPUT centers and
 * *phi (device double, nullable) their cost.  Centroids are summed in FP64
 * in a fixed order and rounded once to FP32. */
int lloyd_step(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
               int64_t n, int32_t d, float* C, int32_t k, int32_t* assign, double* phi, void* ws,
               size_t ws_bytes, void* stream);

/* `iters` Lloyd iterations (Section 1; Section 3.1) in one call, each exactly
 * as lloyd_step computes it, so the result equals `iters` lloyd_step calls
 * bit for bit; X's own preparation (its norms and, in REFINED mode, the
 * screen's operands) is done once for all of them.  C [k x d FP32] is
 * updated in place; assign [n] (nullable) receives the last iteration's
 * assignment (to its input centers) and phi (device, nullable) the cost of
 * each iteration's input centers, phi[0 .. iters-1].  iters = 0 does
 * nothing.  Workspace: kmpar_workspace_size(KMPAR_OP_LLOYD, ...). */
int kmpar_lloyd(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                int64_t n, int32_t d, float* C, int32_t k, int32_t iters, int32_t* assign,
                double* phi, void* ws, size_t ws_bytes, void* stream);

/* k-means++ on all of X (Algorithm 1, the initialisation k-means|| is
 * measured against in Section 4.2): the first center is point Index(n) of
 * Philox tag 1 (as kmpar_init's), then center s = 1 .. k-1 is drawn in
 * proportion to d^2(x, {centers so far}) by the exponential race of
 * KMPAR_OPT_SAMPLING (tag 4, counter (i, s, 0)); each step is one pass over
 * X (FP32 direct-form distances to the newest center, folded into d^2).
 * Output: centers [k x d] FP32 in pick order; picks [k] (device, nullable)
 * their point indices; phi [k] (device, nullable) the cost after each pick,
 * phi[s] = phi_X(first s + 1 centers); stats (device, nullable): phi[0] =
 * psi, n_centers.  If every point lies on a center before k picks, the run
 * stops there with stats->status = KMPAR_E_TOOFEW.  Workspace:
 * kmpar_workspace_size(KMPAR_OP_KMEANSPP, ...). */
int kmpar_kmeanspp(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                   int64_t n, int32_t d, int32_t k, uint64_t seed, float* centers, int32_t* picks,
                   double* phi, void* ws, size_t ws_bytes, kmpar_stats* stats, void* stream);

/* Lloyd's iteration until the centers are stable (Section 1): every
 * iteration assigns each point to its nearest center (as lloyd_step); when
 * the assignment equals the previous iteration's the centers would not move
 * and the call stops, otherwise the centers move to the centroids.  At most
 * max_iters center updates.  *iters (HOST int) receives the number of
 * updates made (max_iters if the assignment never settled); phi [max_iters
 * + 1] (device, nullable) the cost of each assignment's centers, phi[*iters]
 * that of the final ones; assign [n] (device, nullable) the final
 * assignment.  Unlike every other call this one reads a count back to the
 * host once per iteration (it synchronises the stream and cannot be
 * captured in a graph).  Workspace: kmpar_workspace_size(KMPAR_OP_LLOYD). */
int kmpar_lloyd_until_stable(kmpar_ctx* ctx, const void* X, const float* row_scale,
                             kmpar_dtype dtype, int64_t n, int32_t d, float* C, int32_t k,
                             int32_t max_iters, int32_t* iters, int32_t* assign, double* phi,
                             void* ws, size_t ws_bytes, void* stream);

/* One independent clustering instance of kmpar_init_batched (64 bytes). */
typedef struct kmpar_instance {
  const void* X;          /* device: n x d rows, the call's dtype            */
  const float* row_scale; /* device: FP8 row scales, else NULL               */
  float* centers;         /* device: k x d output, pick order                */
  kmpar_stats* stats;     /* device, nullable                                */
  int64_t n;
  int32_t d;
  int32_t k;
  double ell;
  int32_t rounds;
  int32_t reserved;
} kmpar_instance;

/* Workspace bytes of kmpar_init_batched for these instances (host array). */
int kmpar_workspace_size_batched(const kmpar_ctx* ctx, const kmpar_instance* inst_host,
                                 int32_t count, kmpar_dtype dtype, size_t* bytes_out);

/* Algorithm 2 for `count` independent instances in grouped launches: every
 * kernel covers all instances at once (work lists built on the device), so
 * the whole batch is a fixed sequence of about 8 + 9*rounds launches.
 * Instance i draws from Philox with inst = i (same keys and counters as
 * kmpar_init otherwise), so each instance is reproducible on its own.
 * `inst_host` and `inst_dev` hold the same table: the host copy sizes the
 * launches, the device copy is what the kernels read (the library copies
 * nothing between host and device).  All instances share `dtype`; the
 * distance pass is the FP32 direct form whatever the context's mode (a
 * REFINED context gives the same results, as its decisions equal PLAIN's).
 * Limits per instance as for kmpar_init; rounds must be equal across the
 * batch.  Per-instance stats are written when inst[i].stats is not NULL.
 * `traces_dev` (nullable) is a DEVICE array of `count` kmpar_trace records
 * whose non-NULL fields receive instance i's candidates, weights, picks,
 * assignment and D^2 as kmpar_init's trace does. */
int kmpar_init_batched(kmpar_ctx* ctx, const kmpar_instance* inst_host,
                       const kmpar_instance* inst_dev, int32_t count, kmpar_dtype dtype,
                       uint64_t seed, void* ws, size_t ws_bytes, const kmpar_trace* traces_dev,
                       void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KMPAR_H_ */
