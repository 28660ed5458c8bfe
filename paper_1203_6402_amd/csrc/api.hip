// Host side of the kmpar C ABI: argument validation (before any HIP call),
// workspace layout, and the launch sequence of each call.  No call allocates
// device memory or synchronises the host.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/kmpar.h"
#include "kernels.hpp"

namespace {
// One timed launch of a distance kernel (see kmpar_profile_enable).
struct ProfRec {
  int slot;
  hipEvent_t a, b;
  int64_t npts;          // points processed (when npts_dev == nullptr)
  const int* npts_dev;   // device count of points processed (nullable)
  const int* rs_dev;     // device rs pair: m = rs[1] - rs[0] (nullable)
  int m_host;
};
}  // namespace

struct kmpar_ctx {
  int device = -1;
  void* scratch = nullptr;  // this device's copy of the fixed scratch (kmpar_cost_noalloc)
  int num_cu = 1;
  kmpar_mode mode = KMPAR_MODE_PLAIN_FP32;
  std::string err;
  bool prof = false;
  int recl_path = 0;  // KMPAR_OPT_RECLUSTER_PATH
  int sampling = 0;   // KMPAR_OPT_SAMPLING
  kmpar::BatchTuner tuner;  // KMPAR_OPT_BATCH_AUTOTUNE and its choices
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
};

namespace {

using namespace kmpar;

constexpr int kMaxD = 256;
constexpr int kMaxK = 16384;
// Below these candidate counts the direct form is at least as fast.
constexpr double kScreenMinEll = 32.0;
constexpr int kScreenMinM = 32;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int set_err(kmpar_ctx* ctx, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int set_err(kmpar_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int64_t cap_round_of(int64_t n, double ell) { return cap_round_hd(n, ell); }

// Sequential carve-up of the caller's workspace.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    T* p = base ? (T*)(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

struct InitLayout {
  float* D2;
  int* A;
  float* S;  // second-smallest distance per point (flagged argmins)
  double* phi_part;
  int* cnt;
  uint64_t* keep;  // per-round masks of kept points, one bit per point
  int* rs;
  int* scan_total;
  int* cand_point;
  float* Call;
  float* CallT;
  int* w;
  double* rpart;  // recluster partial slots [k][G]
  double* udraw;  // recluster draws [k]
  float* prow;    // recluster row slots [k][DP]
  int* picks;
  kmpar_stats* st;
  float* norms;
  int* list;
  int* list_len;
  int4* rescan_part;  // slice winners of a split rescan
  void* B;
  float* ncg;
  float* scg;
  int* cperm;     // the round's candidates in norm order (tile positions)
  float2* tnr;    // each tile's norm interval
  void* Apre;
  ExactWs ex;     // exact-ell rounds only
  size_t bytes;
};

// Bytes of prepared A operands for the screen of this dtype (0 if unused).
size_t a_bytes(kmpar_dtype dt, bool rows, int64_t n, int d) {
  if (!screen_supported(dt, rows, d)) return 0;
  const int sp = screen_split(dt, rows);
  if (screen_a_direct(dt, sp, d)) return 0;
  return screen_a_bytes((int)n, screen_ksteps(sp, d));
}

InitLayout init_layout(void* ws, int64_t n, int d, int k, double ell, int rounds, kmpar_dtype dt,
                       bool exact) {
  const int DP = padded_dim(d);
  const int64_t capT = 1 + (int64_t)rounds * cap_round_of(n, ell);
  Carver c(ws);
  InitLayout L;
  L.D2 = c.take<float>(n);
  L.A = c.take<int>(n);
  L.S = c.take<float>(n);
  L.phi_part = c.take<double>((n + kPhiChunk - 1) / kPhiChunk);
  L.cnt = c.take<int>((n + kDrawChunk - 1) / kDrawChunk + 1);
  L.keep = c.take<uint64_t>((n + kDrawChunk - 1) / kDrawChunk * (kDrawChunk / 64));
  L.rs = c.take<int>(rounds + 2);
  L.scan_total = c.take<int>(4);
  L.cand_point = c.take<int>(capT);
  L.Call = c.take<float>(capT * DP);
  L.CallT = c.take<float>(capT * d);
  L.w = c.take<int>(capT);
  // one partial per (pick, block) and one row per pick: the recluster never
  // reuses a slot (the grid at launch has at most this many blocks)
  ReclPlan plan{kReclMaxBlocks, 1, false, 0};
  const int G_max = recluster_plan((int)capT, DP, kReclMaxBlocks, false, &plan) ? plan.G : kReclMaxBlocks;
  L.rpart = c.take<double>((size_t)k * G_max);
  L.udraw = c.take<double>(k);
  L.prow = c.take<float>((size_t)k * DP);
  L.picks = c.take<int>(k);
  L.st = c.take<kmpar_stats>(1);
  const int tiles = (int)((cap_round_of(n, ell) + 15) / 16);
  L.norms = c.take<float>(n);
  L.list = c.take<int>(n);
  L.list_len = c.take<int>(4);
  L.rescan_part = c.take<int4>((size_t)kRescanMaxItems * kRescanPts);
  L.B = c.take<char>(screen_b_bytes(tiles, d));
  L.ncg = c.take<float>((size_t)tiles * 16);
  L.scg = c.take<float>((size_t)tiles * 16);
  L.cperm = c.take<int>((size_t)tiles * 16);
  L.tnr = c.take<float2>((size_t)tiles);
  L.Apre = c.take<char>(a_bytes(dt, true, n, d));
  L.ex = ExactWs{};
  if (exact) {
    L.ex.keys = c.take<unsigned long long>(n);
    L.ex.hist = c.take<int>(exact_hist_bins());
    L.ex.state = c.take<ExactState>(1);
  }
  L.bytes = c.off;
  return L;
}

// Workspace of kmpar_assign_sharded.
struct ShardLayout {
  float* Cpad;
  unsigned long long* packed;
  float* D2;
  double* phi_part;
  size_t bytes;
};

ShardLayout shard_layout(void* ws, int64_t n, int d, int64_t m) {
  Carver c(ws);
  ShardLayout L{};
  L.Cpad = c.take<float>((size_t)m * padded_dim(d));
  L.packed = c.take<unsigned long long>(n);
  L.D2 = c.take<float>(n);
  L.phi_part = c.take<double>((n + kPhiChunk - 1) / kPhiChunk);
  L.bytes = c.off;
  return L;
}

constexpr int64_t kMaxShardedM = (int64_t)1 << 24;
constexpr int kMaxShards = 256;

// The exact-ell rounds of a context (sized in its workspace); a null
// context sizes for them.
bool ctx_exact(const kmpar_ctx* ctx) { return !ctx || ctx->sampling == 1; }

// Workspace of kmpar_kmeanspp.
struct KppLayout {
  KppWs w;
  int* picks;
  kmpar_stats* st;
  size_t bytes;
};

KppLayout kpp_layout(void* ws, int64_t n, int d, int k) {
  Carver c(ws);
  KppLayout L{};
  const int64_t nb = (n + 63) / 64;
  L.w.D2 = c.take<float>(n);
  L.w.pkey = c.take<unsigned long long>(nb);
  L.w.pidx = c.take<int>(nb);
  L.w.pphi = c.take<double>(nb);
  L.w.crow = c.take<float>(d);
  L.w.stop = c.take<int>(4);
  L.w.qkey = c.take<unsigned long long>(kKppQ);
  L.w.qidx = c.take<int>(kKppQ);
  L.w.qphi = c.take<double>(kKppQ);
  L.picks = c.take<int>(k);
  L.st = c.take<kmpar_stats>(1);
  L.bytes = c.off;
  return L;
}

struct AssignLayout {
  float* D2;
  int* A;
  double* phi_part;
  double* phi_tmp;
  float* Cpad;
  LloydWs lw;
  int* A2;       // Lloyd until stable: the previous iteration's assignment
  int* changed;  // and the count of points whose assignment changed
  float* norms;
  int* list;
  int* list_len;
  int4* rescan_part;  // slice winners of a split rescan
  void* B;
  float* ncg;
  float* scg;
  void* Apre;
  size_t bytes;
};

// refined: the context screens assignment passes (REFINED mode), so the
// screen's buffers (norms, list, operands) are carved as well.
AssignLayout assign_layout(void* ws, int64_t n, int d, int k, kmpar_op op, kmpar_dtype dt,
                           bool refined) {
  const int DP = padded_dim(d);
  Carver c(ws);
  AssignLayout L{};
  L.D2 = c.take<float>(n);
  L.A = c.take<int>(n);
  L.phi_part = c.take<double>((n + kPhiChunk - 1) / kPhiChunk);
  L.phi_tmp = c.take<double>(1);
  L.Cpad = c.take<float>((size_t)k * DP);
  if (op == KMPAR_OP_LLOYD) {
    const int64_t nbs = (n + kSortChunk - 1) / kSortChunk;
    const int64_t Lt = (int64_t)(k + 1) * nbs;  // keys 0 .. k (k: no valid center)
    L.lw.bcnt = c.take<int>(Lt);
    L.lw.scan_tmp = c.take<int>((Lt + kScanTile - 1) / kScanTile + 1);
    L.lw.sorted = c.take<int>(n);
    L.lw.cstart = c.take<int>(k + 1);
    L.lw.coff = c.take<int>(k + 1);
    L.lw.part = c.take<double>(((n + kSegChunk - 1) / kSegChunk + k) * (int64_t)d);
    L.A2 = c.take<int>(n);
    L.changed = c.take<int>(4);
  }
  if (refined && screen_supported(dt, false, d)) {
    const int tiles = (k + 15) / 16;
    L.norms = c.take<float>(n);
    L.list = c.take<int>(n);
    L.list_len = c.take<int>(4);
    L.rescan_part = c.take<int4>((size_t)kRescanMaxItems * kRescanPts);
    L.B = c.take<char>(screen_b_bytes(tiles, d));
    L.ncg = c.take<float>((size_t)tiles * 16);
    L.scg = c.take<float>((size_t)tiles * 16);
    L.Apre = c.take<char>(a_bytes(dt, false, n, d));
  }
  L.bytes = c.off;
  return L;
}

// Whether assignment passes of this context screen (sizes its workspace
// for it); a null context sizes for the screen.
bool ctx_refined(const kmpar_ctx* ctx) { return !ctx || ctx->mode == KMPAR_MODE_REFINED; }

int check_common(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dt, int64_t n,
                 int32_t d) {
  if (dt != KMPAR_F32 && dt != KMPAR_BF16 && dt != KMPAR_FP8_E4M3)
    return set_err(ctx, KMPAR_E_INVAL, "unknown dtype %d", (int)dt);
  if (n < 1 || n >= (int64_t)1 << 31) return set_err(ctx, KMPAR_E_INVAL, "n=%lld out of range", (long long)n);
  if (d < 1 || d > kMaxD) return set_err(ctx, KMPAR_E_INVAL, "d=%d out of range [1,%d]", d, kMaxD);
  if (!X || !aligned16(X)) return set_err(ctx, KMPAR_E_INVAL, "X is NULL or not 16-byte aligned");
  if (dt == KMPAR_FP8_E4M3) {
    if (!row_scale || !aligned16(row_scale))
      return set_err(ctx, KMPAR_E_INVAL, "FP8 input needs a 16-byte aligned row_scale");
  } else if (row_scale) {
    return set_err(ctx, KMPAR_E_INVAL, "row_scale is only valid with KMPAR_FP8_E4M3");
  }
  return KMPAR_OK;
}

bool ell_ok(double ell) { return isfinite(ell) && ell > 0.0; }

// Makes ctx->device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  hipError_t e = hipSuccess;
  explicit DeviceGuard(int dev) {
    e = hipGetDevice(&prev);
    if (e != hipSuccess) return;
    if (prev != dev) e = hipSetDevice(dev);
    ok = (e == hipSuccess);
  }
  ~DeviceGuard() {
    if (ok && prev >= 0) {
      int cur = -1;
      if (hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
  }
};

int hip_fail(kmpar_ctx* ctx, hipError_t e, const char* where) {
  return set_err(ctx, KMPAR_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define KMPAR_HIP(call)                                       \
  do {                                                        \
    hipError_t _e = (call);                                   \
    if (_e != hipSuccess) return hip_fail(ctx, _e, #call);    \
  } while (0)

hipError_t prof_event(kmpar_ctx* ctx, hipEvent_t* e) {
  if (!ctx->pool.empty()) {
    *e = ctx->pool.back();
    ctx->pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Runs `launch`, bracketed by events when profiling is on.
template <typename F>
hipError_t timed(kmpar_ctx* ctx, int slot, int64_t npts, const int* npts_dev, const int* rs_dev,
                 int m_host, hipStream_t s, F&& launch) {
  if (!ctx->prof) return launch();
  ProfRec r{};
  r.slot = slot;
  hipError_t e;
  if ((e = prof_event(ctx, &r.a)) != hipSuccess) return e;
  if ((e = prof_event(ctx, &r.b)) != hipSuccess) return e;
  if ((e = hipEventRecord(r.a, s)) != hipSuccess) return e;
  if ((e = launch()) != hipSuccess) return e;
  if ((e = hipEventRecord(r.b, s)) != hipSuccess) return e;
  r.npts = npts;
  r.npts_dev = npts_dev;
  r.rs_dev = rs_dev;
  r.m_host = m_host;
  ctx->recs.push_back(r);
  return hipSuccess;
}

// Slots of kmpar_profile_read.
enum { kSlotDirect = 0, kSlotScreen = 1, kSlotRescan = 2, kSlotBatchFold = 3 };

hipError_t timed_fold(kmpar_ctx* ctx, int slot, kmpar_dtype dt, int DP, const FoldArgs& fa,
                      hipStream_t s) {
  return timed(ctx, slot, fa.list ? 0 : fa.n, fa.list ? fa.list_len : nullptr, fa.rs, fa.m_host, s,
               [&] { return launch_fold_direct(dt, DP, fa, s); });
}

// One REFINED distance pass: B operands, screen, direct-form rescan of the
// points the screen listed.  `fa` describes the same pass for the direct form.
// FP8 rows also take the candidates' point ids (cand), whose codes are the
// B operands, and their scales (scg).
hipError_t refined_pass(kmpar_ctx* ctx, kmpar_dtype dt, int split, int DP, const FoldArgs& fa,
                        int max_tiles, const float* norms, const void* Apre, void* B, float* ncg,
                        const int* cand, float* scg, int* list, int* list_len, int4* rpart,
                        int* cperm, float2* tnr, kmpar_stats* st, hipStream_t s) {
  const int KS = screen_ksteps(split, fa.d);
  // A pass of at most kScreenOneGroupMaxTiles tiles tags each tile by its
  // index in the pass (single-group screen); the bound covers the tag.
  const int tag_bits = max_tiles <= kScreenOneGroupMaxTiles ? screen_pass_tag_bits(max_tiles) : 0;
  const float om2g =
      1.0f - 2.0f * screen_g(dt, split, fa.d, tag_bits > 0 ? tag_bits : screen_tag_bits(KS));
  const bool fp8 = dt == KMPAR_FP8_E4M3;
  // The candidates in norm order and each tile's norm interval, for the
  // tile skip of the three-wave single-group screen in passes that keep D
  // (init rounds); other passes keep id order.
  if (!(cperm && tag_bits > 0 && screen_three_waves(KS, true, fp8) && !fa.first)) {
    cperm = nullptr;
    tnr = nullptr;
  }
  if (cperm) {
    hipError_t e0 = launch_cand_sort(fa.C, DP, fa.d, fa.rs, fa.m_host, cperm, tnr, s);
    if (e0 != hipSuccess) return e0;
  }
  hipError_t e = launch_prep_b(dt, split, KS, fa.C, DP, fa.d, fa.rs, fa.m_host, max_tiles, om2g, B,
                               ncg, fa.X, fa.row_scale, fp8 ? cand : nullptr,
                               fp8 ? scg : nullptr, list_len, st, cperm, s);
  if (e != hipSuccess) return e;
  ScreenArgs sa{};
  sa.X = fa.X;
  sa.row_scale = fa.row_scale;
  sa.n = fa.n;
  sa.d = fa.d;
  sa.DP = DP;
  sa.C = fa.C;
  sa.rs = fa.rs;
  sa.m_host = fa.m_host;
  sa.id0_host = fa.id0_host;
  sa.Apre = Apre;
  sa.B = B;
  sa.ncg = ncg;
  sa.scg = fp8 ? scg : nullptr;
  sa.norms = norms;
  sa.oneminus2g = om2g;
  sa.D2 = fa.D2;
  sa.A = fa.A;
  sa.S = fa.S;
  sa.first = fa.first;
  sa.list = list;
  sa.list_len = list_len;
  sa.stats = st;
  sa.tag_bits = tag_bits;
  sa.cperm = cperm;
  sa.tnr = tnr;
  e = timed(ctx, kSlotScreen, fa.n, nullptr, fa.rs, fa.m_host, s,
            [&] { return launch_screen(dt, split, KS, sa, s); });
  if (e != hipSuccess) return e;
  FoldArgs rf = fa;
  rf.list = list;
  rf.list_len = list_len;
  rf.list_cap = fa.n;
  rf.norms = nullptr;
  rf.rpart = rpart;
  return timed(ctx, kSlotRescan, 0, list_len, fa.rs, fa.m_host, s,
               [&] { return launch_rescan(dt, DP, rf, s); });
}

int device_ready(kmpar_ctx* ctx) {
  if (ctx->device < 0) return set_err(ctx, KMPAR_E_NODEVICE, "context has no device");
  return KMPAR_OK;
}

// Fixed device scratch of kmpar_cost_noalloc, for callers that cannot
// allocate: one copy on every GPU the library runs on, held until the
// process ends.  In host code `scratch` only names the symbol; the device
// address of each GPU's copy comes from hipGetSymbolAddress, taken once per
// device when the first context on it is created, and only that address is
// passed to kernels.
constexpr size_t kNoallocBytes = KMPAR_NOALLOC_SCRATCH_BYTES;

}  // namespace

static __device__ __attribute__((aligned(256))) char scratch[KMPAR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The address of `scratch` on device dev (made current here), looked up once.
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    DeviceGuard g(dev);
    if (!g.ok) return g.e;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// kmpar_cost's launch sequence on the workspace ws (validated by the caller).
int cost_run(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype, int64_t n,
             int32_t d, const float* C, int32_t m, double* phi, void* ws, size_t ws_bytes,
             void* stream);

}  // namespace

extern "C" {

int kmpar_create(int hip_device, kmpar_mode mode, kmpar_ctx** out) {
  if (!out) return KMPAR_E_INVAL;
  *out = nullptr;
  if (mode != KMPAR_MODE_PLAIN_FP32 && mode != KMPAR_MODE_REFINED) return KMPAR_E_INVAL;
  if (hip_device < -1) return KMPAR_E_INVAL;
  if (hip_device >= 0) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device >= count) return KMPAR_E_HIP;
  }
  int cu = 1;
  if (hip_device >= 0 &&
      hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess)
    return KMPAR_E_HIP;
  void* scr = nullptr;
  if (hip_device >= 0 && scratch_address(hip_device, &scr) != hipSuccess) return KMPAR_E_HIP;
  kmpar_ctx* c = new kmpar_ctx;
  c->num_cu = cu;
  c->device = hip_device;
  c->mode = mode;
  c->scratch = scr;
  *out = c;
  return KMPAR_OK;
}

void kmpar_destroy(kmpar_ctx* ctx) {
  if (!ctx) return;
  for (auto& r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
}

int kmpar_set_option(kmpar_ctx* ctx, kmpar_option opt, int64_t value) {
  if (!ctx) return KMPAR_E_INVAL;
  switch (opt) {
    case KMPAR_OPT_RECLUSTER_PATH:
      if (value < 0 || value > 3) return set_err(ctx, KMPAR_E_INVAL, "recluster path %lld", (long long)value);
      ctx->recl_path = (int)value;
      return KMPAR_OK;
    case KMPAR_OPT_SAMPLING:
      if (value < 0 || value > 1) return set_err(ctx, KMPAR_E_INVAL, "sampling %lld", (long long)value);
      ctx->sampling = (int)value;
      return KMPAR_OK;
    case KMPAR_OPT_BATCH_AUTOTUNE:
      if (value < 0 || value > 1) return set_err(ctx, KMPAR_E_INVAL, "batch autotune %lld", (long long)value);
      ctx->tuner.enabled = value != 0;
      return KMPAR_OK;
  }
  return set_err(ctx, KMPAR_E_INVAL, "unknown option %d", (int)opt);
}

int kmpar_batch_tiles(const kmpar_ctx* ctx, int32_t* dtype, int32_t* dp, int32_t* cb, int32_t cap,
                      int32_t* count) {
  if (!ctx || !count || cap < 0 || (cap > 0 && (!dtype || !dp || !cb))) return KMPAR_E_INVAL;
  int32_t c = 0;
  for (const auto& kv : ctx->tuner.cb) {
    if (c < cap) {
      dtype[c] = kv.first / 4096;
      dp[c] = kv.first % 4096;
      cb[c] = kv.second;
    }
    ++c;
  }
  *count = c;
  return KMPAR_OK;
}

int kmpar_profile_enable(kmpar_ctx* ctx, int on) {
  if (!ctx) return KMPAR_E_INVAL;
  ctx->prof = on != 0;
  return KMPAR_OK;
}

int kmpar_profile_read(kmpar_ctx* ctx, int slot, int64_t* launches, double* total_ms,
                       double* pairs) {
  if (!ctx || !launches || !total_ms || !pairs) return KMPAR_E_INVAL;
  *launches = 0;
  *total_ms = 0.0;
  *pairs = 0.0;
  if (ctx->recs.empty()) return KMPAR_OK;
  if (ctx->device < 0) return set_err(ctx, KMPAR_E_NODEVICE, "context has no device");
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  std::vector<ProfRec> keep;
  for (auto& r : ctx->recs) {
    if (r.slot != slot) {
      keep.push_back(r);
      continue;
    }
    KMPAR_HIP(hipEventSynchronize(r.b));
    float ms = 0.0f;
    KMPAR_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    int64_t npts = r.npts;
    if (r.npts_dev) {
      int v = 0;
      KMPAR_HIP(hipMemcpy(&v, r.npts_dev, sizeof(int), hipMemcpyDeviceToHost));
      npts = v;
    }
    int64_t m = r.m_host;
    if (r.rs_dev) {
      int v[2] = {0, 0};
      KMPAR_HIP(hipMemcpy(v, r.rs_dev, sizeof v, hipMemcpyDeviceToHost));
      m = v[1] - v[0];
    }
    *launches += 1;
    *total_ms += ms;
    *pairs += (double)npts * (double)m;
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->recs.swap(keep);
  return KMPAR_OK;
}

const char* kmpar_strerror(int status) {
  switch (status) {
    case KMPAR_OK: return "ok";
    case KMPAR_E_INVAL: return "invalid argument";
    case KMPAR_E_WORKSPACE: return "workspace too small";
    case KMPAR_E_HIP: return "HIP runtime error";
    case KMPAR_E_TOOFEW: return "fewer than k distinct candidates";
    case KMPAR_E_OVERFLOW: return "a round exceeded the candidate capacity";
    case KMPAR_E_NODEVICE: return "context has no device";
  }
  return "unknown status";
}

const char* kmpar_last_error(const kmpar_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

size_t kmpar_sizeof_stats(void) { return sizeof(kmpar_stats); }

int kmpar_max_candidates(int64_t n, double ell, int32_t rounds, int64_t* out) {
  if (!out || n < 1 || !ell_ok(ell) || rounds < 0 || rounds > KMPAR_MAX_ROUNDS)
    return KMPAR_E_INVAL;
  *out = 1 + (int64_t)rounds * cap_round_of(n, ell);
  return KMPAR_OK;
}

int kmpar_workspace_size(const kmpar_ctx* cctx, kmpar_op op, int64_t n, int32_t d, int32_t k,
                         double ell, int32_t rounds, kmpar_dtype dtype, size_t* bytes_out) {
  kmpar_ctx* ctx = const_cast<kmpar_ctx*>(cctx);
  if (!bytes_out) return set_err(ctx, KMPAR_E_INVAL, "bytes_out is NULL");
  if (dtype != KMPAR_F32 && dtype != KMPAR_BF16 && dtype != KMPAR_FP8_E4M3)
    return set_err(ctx, KMPAR_E_INVAL, "unknown dtype");
  if (n < 1 || n >= (int64_t)1 << 31 || d < 1 || d > kMaxD || k < 1 ||
      k > (op == KMPAR_OP_ASSIGN_SHARDED ? kMaxShardedM : kMaxK))
    return set_err(ctx, KMPAR_E_INVAL, "size out of range");
  switch (op) {
    case KMPAR_OP_INIT: {
      if (k > n || !ell_ok(ell) || rounds < 0 || rounds > KMPAR_MAX_ROUNDS)
        return set_err(ctx, KMPAR_E_INVAL, "k, ell or rounds out of range");
      const int64_t capT = 1 + (int64_t)rounds * cap_round_of(n, ell);
      if (capT >= (int64_t)1 << 31) return set_err(ctx, KMPAR_E_INVAL, "candidate capacity too large");
      if (ctx && ctx->sampling == 1 && (ell != floor(ell) || ell > INT32_MAX))
        return set_err(ctx, KMPAR_E_INVAL, "exact-ell rounds need an integer ell");
      *bytes_out = init_layout(nullptr, n, d, k, ell, rounds, dtype, ctx_exact(ctx)).bytes;
      return KMPAR_OK;
    }
    case KMPAR_OP_ASSIGN_SHARDED:
      *bytes_out = shard_layout(nullptr, n, d, k).bytes;
      return KMPAR_OK;
    case KMPAR_OP_KMEANSPP:
      if (k > n) return set_err(ctx, KMPAR_E_INVAL, "k=%d > n", k);
      *bytes_out = kpp_layout(nullptr, n, d, k).bytes;
      return KMPAR_OK;
    case KMPAR_OP_COST:
    case KMPAR_OP_ASSIGN:
    case KMPAR_OP_LLOYD:
      *bytes_out = assign_layout(nullptr, n, d, k, op, dtype, ctx_refined(ctx)).bytes;
      return KMPAR_OK;
  }
  return set_err(ctx, KMPAR_E_INVAL, "unknown op");
}

int kmpar_init(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype, int64_t n,
               int32_t d, int32_t k, double ell, int32_t rounds, uint64_t seed, float* centers,
               void* ws, size_t ws_bytes, kmpar_stats* stats, const kmpar_trace* trace,
               void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  int rc = check_common(ctx, X, row_scale, dtype, n, d);
  if (rc) return rc;
  if (k < 1 || k > n || k > kMaxK) return set_err(ctx, KMPAR_E_INVAL, "k=%d out of range", k);
  if (!ell_ok(ell)) return set_err(ctx, KMPAR_E_INVAL, "ell must be finite and > 0");
  if (rounds < 0 || rounds > KMPAR_MAX_ROUNDS)
    return set_err(ctx, KMPAR_E_INVAL, "rounds=%d out of range", rounds);
  if (!centers || !aligned16(centers)) return set_err(ctx, KMPAR_E_INVAL, "centers NULL/misaligned");
  if (stats && ((uintptr_t)stats & 7u)) return set_err(ctx, KMPAR_E_INVAL, "stats misaligned");
  if (!ws) return set_err(ctx, KMPAR_E_INVAL, "workspace is NULL");
  size_t need = 0;
  rc = kmpar_workspace_size(ctx, KMPAR_OP_INIT, n, d, k, ell, rounds, dtype, &need);
  if (rc) return rc;
  if (ws_bytes < need)
    return set_err(ctx, KMPAR_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  // The candidate capacity must fit an int, and step 8 must fit the CUs
  // (rows in LDS or in global memory) unless the one-workgroup path is chosen.
  const int64_t capT64 = 1 + (int64_t)rounds * cap_round_of(n, ell);
  if (capT64 > INT32_MAX)
    return set_err(ctx, KMPAR_E_INVAL, "candidate capacity %lld exceeds 2^31 - 1",
                   (long long)capT64);
  ReclPlan recl{};
  const bool recl_ok =
      recluster_plan((int)capT64, padded_dim(d), ctx->device >= 0 ? ctx->num_cu : kReclMaxBlocks,
                     ctx->recl_path == 3, &recl);
  if (!recl_ok && !(ctx->recl_path == 1 && recluster_block_lds((int)capT64, k) <= kReclBlockLdsMax))
    return set_err(ctx, KMPAR_E_INVAL, "candidate capacity %lld too large for the recluster",
                   (long long)capT64);
  if ((rc = device_ready(ctx))) return rc;

  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int N = (int)n, DP = padded_dim(d);
  const int cap_round = (int)cap_round_of(n, ell);
  const int capT = (int)capT64;
  InitLayout L = init_layout(ws, n, d, k, ell, rounds, dtype, ctx_exact(ctx));
  const bool exact = ctx->sampling == 1;
  kmpar_stats* st = stats ? stats : L.st;
  const uint64_t inst = 0;

  // Steps 1-2: first center, D2 against it, psi.
  KMPAR_HIP(launch_first(N, seed, inst, L.cand_point, L.rs, st, s));
  KMPAR_HIP(launch_fill_i32(reinterpret_cast<int*>(L.S), 0x7F800000, N, s));  // +inf
  KMPAR_HIP(launch_gather(dtype, X, row_scale, d, DP, L.cand_point, L.rs, 0, 1, L.Call, L.CallT,
                          capT, s));
  FoldArgs fa{};
  fa.X = X;
  fa.row_scale = row_scale;
  fa.n = N;
  fa.d = d;
  fa.C = L.Call;
  fa.D2 = L.D2;
  fa.A = L.A;
  fa.S = L.S;
  fa.rs = L.rs;
  fa.first = 1;
  // The REFINED screen runs on the rounds (m_t ~ ell candidates); the first
  // pass has m = 1 and stays in direct form, where it also writes ||x||^2.
  const int split = screen_split(dtype, true);
  const bool refined = ctx->mode == KMPAR_MODE_REFINED && screen_supported(dtype, true, d) &&
                       ell >= kScreenMinEll;
  // One coalesced read of X: D2 against the first center, and for REFINED
  // ||x||^2 and (unless X rows are the operands) the screen's A operands.
  const bool prep = refined && !screen_a_direct(dtype, split, d);
  const void* Apre = prep ? L.Apre : nullptr;
  KMPAR_HIP(timed(ctx, kSlotDirect, N, nullptr, L.rs, 1, s, [&] {
    return launch_first_pass(dtype, split, refined ? screen_ksteps(split, d) : 1, prep, X,
                             row_scale, N, d, DP, L.Call, L.rs, L.D2, L.A,
                             refined ? L.norms : nullptr, prep ? L.Apre : nullptr, s);
  }));
  KMPAR_HIP(launch_phi(L.D2, N, L.phi_part, &st->phi[0], s));
  if (refined) KMPAR_HIP(launch_fill_i32(L.list_len, 0, 1, s));
  if (exact) KMPAR_HIP(launch_fill_i32(L.ex.hist, 0, exact_hist_bins(), s));
  // Steps 3-6: rounds.
  fa.first = 0;
  for (int t = 1; t <= rounds; ++t) {
    if (exact)
      KMPAR_HIP(launch_exact_round(L.D2, N, (int)ell, seed, t, inst, fp32_flag_band(d), L.ex, L.cnt,
                                   L.keep, L.scan_total, L.rs, cap_round, L.cand_point, st, s));
    else
      KMPAR_HIP(launch_draw(L.D2, N, &st->phi[t - 1], ell, seed, t, inst, fp32_flag_band(d), L.cnt,
                            L.keep, L.scan_total, L.rs, cap_round, L.cand_point, st, s));
    KMPAR_HIP(launch_gather(dtype, X, row_scale, d, DP, L.cand_point, L.rs, t, cap_round, L.Call,
                            L.CallT, capT, s));
    fa.rs = L.rs + t;
    if (refined) {
      KMPAR_HIP(refined_pass(ctx, dtype, split, DP, fa, (cap_round + 15) / 16, L.norms, Apre, L.B,
                             L.ncg, L.cand_point, L.scg, L.list, L.list_len, L.rescan_part, L.cperm,
                             L.tnr, st, s));
    } else {
      KMPAR_HIP(timed_fold(ctx, kSlotDirect, dtype, DP, fa, s));
    }
    KMPAR_HIP(launch_phi(L.D2, N, L.phi_part, &st->phi[t], s));
  }
  if (refined) KMPAR_HIP(launch_list_reset(L.list_len, st, s));
  KMPAR_HIP(launch_finish_rounds(L.rs, rounds, st, s));
  KMPAR_HIP(launch_flag_argmins(L.D2, L.S, N, fp32_flag_band(d), st, s));
  // Step 7: weights.
  KMPAR_HIP(launch_hist(L.A, N, L.w, capT, ctx->num_cu, s));
  // Step 8: weighted k-means++.
  int* picks = (trace && trace->center_cand) ? trace->center_cand : L.picks;
  // Automatic: several workgroups (measured faster for a single instance at
  // the benchmark shapes: the one-workgroup pick loop is bound by its
  // 1024-thread FP64 scan and barriers); one workgroup only on request.
  const bool one_wg =
      !recl_ok || (ctx->recl_path == 1 && recluster_block_lds(capT, k) <= kReclBlockLdsMax);
  if (one_wg) {
    KMPAR_HIP(launch_recluster_block(L.CallT, capT, d, L.w, L.rs + rounds + 1, k, seed, inst,
                                     picks, centers, st, fp32_flag_band(d), s));
  } else {
    KMPAR_HIP(launch_recluster(L.Call, DP, d, L.w, L.rs + rounds + 1, k, seed, inst, recl,
                               L.udraw, L.rpart, L.prow, picks, centers, st, fp32_flag_band(d), s));
  }
  if (trace) {
    if (trace->cand_point) KMPAR_HIP(launch_copy_i32(L.cand_point, trace->cand_point, capT, s));
    if (trace->cand_weight) KMPAR_HIP(launch_copy_i32(L.w, trace->cand_weight, capT, s));
    if (trace->assign) KMPAR_HIP(launch_copy_i32(L.A, trace->assign, N, s));
    if (trace->d2) KMPAR_HIP(launch_copy_i32((const int*)L.D2, (int*)trace->d2, N, s));
  }
  return KMPAR_OK;
}

static int assign_common(kmpar_ctx* ctx, kmpar_op op, const void* X, const float* row_scale,
                         kmpar_dtype dtype, int64_t n, int32_t d, const float* C, int32_t m,
                         void* ws, size_t ws_bytes, AssignLayout* L, FoldArgs* fa) {
  int rc = check_common(ctx, X, row_scale, dtype, n, d);
  if (rc) return rc;
  if (m < 1 || m > kMaxK) return set_err(ctx, KMPAR_E_INVAL, "number of centers %d out of range", m);
  if (!C || !aligned16(C)) return set_err(ctx, KMPAR_E_INVAL, "C NULL/misaligned");
  if (!ws) return set_err(ctx, KMPAR_E_INVAL, "workspace is NULL");
  size_t need = 0;
  rc = kmpar_workspace_size(ctx, op, n, d, m, 1.0, 0, dtype, &need);
  if (rc) return rc;
  if (ws_bytes < need)
    return set_err(ctx, KMPAR_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  if ((rc = device_ready(ctx))) return rc;
  *L = assign_layout(ws, n, d, m, op, dtype, ctx_refined(ctx));
  *fa = FoldArgs{};
  fa->X = X;
  fa->row_scale = row_scale;
  fa->n = (int)n;
  fa->d = d;
  fa->C = L->Cpad;
  fa->rs = nullptr;
  fa->m_host = m;
  fa->id0_host = 0;
  fa->D2 = L->D2;
  fa->A = L->A;
  fa->first = 1;
  return KMPAR_OK;
}

// Assignment pass against m FP32 centers (first = 1), REFINED when possible.
// prepared: L.norms (and L.Apre) already hold X's norms and A operands from
// an earlier pass of the same call.
static int assign_pass(kmpar_ctx* ctx, kmpar_dtype dtype, const AssignLayout& L, const FoldArgs& fa,
                       int m, hipStream_t s, bool prepared = false) {
  const int d = fa.d, DP = padded_dim(d);
  if (ctx->mode == KMPAR_MODE_REFINED && screen_supported(dtype, false, d) && m >= kScreenMinM) {
    const int split = screen_split(dtype, false);
    KMPAR_HIP(launch_fill_i32(L.list_len, 0, 1, s));
    const void* Apre = nullptr;
    if (!screen_a_direct(dtype, split, d)) {  // one read of X: norms and A operands
      if (!prepared)
        KMPAR_HIP(launch_prep_a(dtype, split, screen_ksteps(split, d), fa.X, fa.row_scale, fa.n, d,
                                L.norms, L.Apre, s));
      Apre = L.Apre;
    } else if (!prepared) {
      KMPAR_HIP(launch_rownorm(dtype, fa.X, fa.row_scale, fa.n, d, L.norms, s));
    }
    KMPAR_HIP(refined_pass(ctx, dtype, split, DP, fa, (m + 15) / 16, L.norms, Apre, L.B, L.ncg,
                           nullptr, L.scg, L.list, L.list_len, L.rescan_part, nullptr, nullptr,
                           nullptr, s));
  } else {
    KMPAR_HIP(timed_fold(ctx, kSlotDirect, dtype, DP, fa, s));
  }
  return KMPAR_OK;
}

int kmpar_cost(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype, int64_t n,
               int32_t d, const float* C, int32_t m, double* phi, void* ws, size_t ws_bytes,
               void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  if (!phi || ((uintptr_t)phi & 7u)) return set_err(ctx, KMPAR_E_INVAL, "phi NULL/misaligned");
  return cost_run(ctx, X, row_scale, dtype, n, d, C, m, phi, ws, ws_bytes, stream);
}

int kmpar_cost_noalloc(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                       int64_t n, int32_t d, const float* C, int32_t m, double* phi,
                       void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  if (!phi || ((uintptr_t)phi & 7u)) return set_err(ctx, KMPAR_E_INVAL, "phi NULL/misaligned");
  int rc = check_common(ctx, X, row_scale, dtype, n, d);
  if (rc) return rc;
  if (m < 1 || m > kMaxK) return set_err(ctx, KMPAR_E_INVAL, "number of centers %d out of range", m);
  size_t need = 0;
  rc = kmpar_workspace_size(ctx, KMPAR_OP_COST, n, d, m, 1.0, 0, dtype, &need);
  if (rc) return rc;
  if (need > kNoallocBytes)
    return set_err(ctx, KMPAR_E_WORKSPACE,
                   "kmpar_cost_noalloc needs %zu bytes of scratch here, more than its fixed %zu "
                   "(call kmpar_cost with a workspace, or a PLAIN_FP32 context)",
                   need, kNoallocBytes);
  if ((rc = device_ready(ctx))) return rc;
  if (!ctx->scratch) return set_err(ctx, KMPAR_E_HIP, "no scratch address for device %d", ctx->device);
  // The same launches as kmpar_cost on the fixed scratch; no event timing
  // (events are created on demand), so nothing here allocates.
  const bool prof = ctx->prof;
  ctx->prof = false;
  rc = cost_run(ctx, X, row_scale, dtype, n, d, C, m, phi, ctx->scratch, kNoallocBytes, stream);
  ctx->prof = prof;
  return rc;
}

}  // extern "C"

namespace {

int cost_run(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype, int64_t n,
             int32_t d, const float* C, int32_t m, double* phi, void* ws, size_t ws_bytes,
             void* stream) {
  AssignLayout L;
  FoldArgs fa;
  int rc = assign_common(ctx, KMPAR_OP_COST, X, row_scale, dtype, n, d, C, m, ws, ws_bytes, &L, &fa);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  KMPAR_HIP(launch_pad_rows(C, m, d, padded_dim(d), L.Cpad, s));
  if ((rc = assign_pass(ctx, dtype, L, fa, m, s))) return rc;
  KMPAR_HIP(launch_phi(L.D2, (int)n, L.phi_part, phi, s));
  return KMPAR_OK;
}

}  // namespace

extern "C" {

int kmpar_assign(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                 int64_t n, int32_t d, const float* C, int32_t m, int32_t* assign, float* d2,
                 void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  if (!assign || !aligned16(assign)) return set_err(ctx, KMPAR_E_INVAL, "assign NULL/misaligned");
  if (d2 && !aligned16(d2)) return set_err(ctx, KMPAR_E_INVAL, "d2 misaligned");
  AssignLayout L;
  FoldArgs fa;
  int rc = assign_common(ctx, KMPAR_OP_ASSIGN, X, row_scale, dtype, n, d, C, m, ws, ws_bytes, &L, &fa);
  if (rc) return rc;
  fa.A = assign;
  if (d2) fa.D2 = d2;
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  KMPAR_HIP(launch_pad_rows(C, m, d, padded_dim(d), L.Cpad, s));
  if ((rc = assign_pass(ctx, dtype, L, fa, m, s))) return rc;
  return KMPAR_OK;
}

int lloyd_step(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype, int64_t n,
               int32_t d, float* C, int32_t k, int32_t* assign, double* phi, void* ws,
               size_t ws_bytes, void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  if (assign && !aligned16(assign)) return set_err(ctx, KMPAR_E_INVAL, "assign misaligned");
  if (phi && ((uintptr_t)phi & 7u)) return set_err(ctx, KMPAR_E_INVAL, "phi misaligned");
  if (k > n) return set_err(ctx, KMPAR_E_INVAL, "k=%d > n", k);
  AssignLayout L;
  FoldArgs fa;
  int rc = assign_common(ctx, KMPAR_OP_LLOYD, X, row_scale, dtype, n, d, C, k, ws, ws_bytes, &L, &fa);
  if (rc) return rc;
  if (assign) fa.A = assign;
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  KMPAR_HIP(launch_pad_rows(C, k, d, padded_dim(d), L.Cpad, s));
  if ((rc = assign_pass(ctx, dtype, L, fa, k, s))) return rc;
  if (phi) KMPAR_HIP(launch_phi(L.D2, (int)n, L.phi_part, phi, s));
  KMPAR_HIP(launch_lloyd_update(dtype, X, row_scale, (int)n, d, fa.A, k, C, L.lw, s));
  return KMPAR_OK;
}

int kmpar_lloyd(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                int64_t n, int32_t d, float* C, int32_t k, int32_t iters, int32_t* assign,
                double* phi, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  if (iters < 0) return set_err(ctx, KMPAR_E_INVAL, "iters=%d < 0", iters);
  if (assign && !aligned16(assign)) return set_err(ctx, KMPAR_E_INVAL, "assign misaligned");
  if (phi && ((uintptr_t)phi & 7u)) return set_err(ctx, KMPAR_E_INVAL, "phi misaligned");
  if (k > n) return set_err(ctx, KMPAR_E_INVAL, "k=%d > n", k);
  AssignLayout L;
  FoldArgs fa;
  int rc = assign_common(ctx, KMPAR_OP_LLOYD, X, row_scale, dtype, n, d, C, k, ws, ws_bytes, &L, &fa);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  for (int it = 0; it < iters; ++it) {
    FoldArgs fi = fa;
    if (assign && it == iters - 1) fi.A = assign;  // the last assignment goes to the caller
    KMPAR_HIP(launch_pad_rows(C, k, d, padded_dim(d), L.Cpad, s));
    if ((rc = assign_pass(ctx, dtype, L, fi, k, s, it > 0))) return rc;
    if (phi) KMPAR_HIP(launch_phi(L.D2, (int)n, L.phi_part, phi + it, s));
    KMPAR_HIP(launch_lloyd_update(dtype, X, row_scale, (int)n, d, fi.A, k, C, L.lw, s));
  }
  return KMPAR_OK;
}

int kmpar_kmeanspp(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                   int64_t n, int32_t d, int32_t k, uint64_t seed, float* centers, int32_t* picks,
                   double* phi, void* ws, size_t ws_bytes, kmpar_stats* stats, void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  int rc = check_common(ctx, X, row_scale, dtype, n, d);
  if (rc) return rc;
  if (k < 1 || k > n || k > kMaxK) return set_err(ctx, KMPAR_E_INVAL, "k=%d out of range", k);
  if (!centers || !aligned16(centers)) return set_err(ctx, KMPAR_E_INVAL, "centers NULL/misaligned");
  if (picks && !aligned16(picks)) return set_err(ctx, KMPAR_E_INVAL, "picks misaligned");
  if (phi && ((uintptr_t)phi & 7u)) return set_err(ctx, KMPAR_E_INVAL, "phi misaligned");
  if (stats && ((uintptr_t)stats & 7u)) return set_err(ctx, KMPAR_E_INVAL, "stats misaligned");
  if (!ws) return set_err(ctx, KMPAR_E_INVAL, "workspace is NULL");
  size_t need = 0;
  rc = kmpar_workspace_size(ctx, KMPAR_OP_KMEANSPP, n, d, k, 1.0, 0, dtype, &need);
  if (rc) return rc;
  if (ws_bytes < need)
    return set_err(ctx, KMPAR_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  if ((rc = device_ready(ctx))) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  KppLayout L = kpp_layout(ws, n, d, k);
  KMPAR_HIP(launch_kmeanspp(dtype, X, row_scale, (int)n, d, k, seed, 0, L.w, picks ? picks : L.picks,
                            centers, phi, stats ? stats : L.st, s));
  return KMPAR_OK;
}

int kmpar_assign_sharded(kmpar_ctx* ctx, const void* X, const float* row_scale, kmpar_dtype dtype,
                         int64_t n, int32_t d, const float* C, int32_t m, int32_t shards,
                         int32_t* assign, float* d2, double* phi, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  int rc = check_common(ctx, X, row_scale, dtype, n, d);
  if (rc) return rc;
  if (m < 1 || m > kMaxShardedM)
    return set_err(ctx, KMPAR_E_INVAL, "number of centers %d out of range [1, 2^24]", m);
  if (shards < 1 || shards > kMaxShards || shards > m)
    return set_err(ctx, KMPAR_E_INVAL, "shards=%d out of range [1, min(m, %d)]", shards, kMaxShards);
  if (!C || !aligned16(C)) return set_err(ctx, KMPAR_E_INVAL, "C NULL/misaligned");
  if (!assign || !aligned16(assign)) return set_err(ctx, KMPAR_E_INVAL, "assign NULL/misaligned");
  if (d2 && !aligned16(d2)) return set_err(ctx, KMPAR_E_INVAL, "d2 misaligned");
  if (phi && ((uintptr_t)phi & 7u)) return set_err(ctx, KMPAR_E_INVAL, "phi misaligned");
  if (!ws) return set_err(ctx, KMPAR_E_INVAL, "workspace is NULL");
  size_t need = 0;
  rc = kmpar_workspace_size(ctx, KMPAR_OP_ASSIGN_SHARDED, n, d, m, 1.0, 0, dtype, &need);
  if (rc) return rc;
  if (ws_bytes < need)
    return set_err(ctx, KMPAR_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  if ((rc = device_ready(ctx))) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int DP = padded_dim(d);
  ShardLayout L = shard_layout(ws, n, d, m);
  float* D2 = d2 ? d2 : L.D2;
  KMPAR_HIP(launch_pad_rows(C, m, d, DP, L.Cpad, s));
  // every packed minimum starts at all-ones (above any distance and id)
  KMPAR_HIP(launch_fill_i32(reinterpret_cast<int*>(L.packed), -1, 2 * n, s));
  FoldArgs fa{};
  fa.X = X;
  fa.row_scale = row_scale;
  fa.n = (int)n;
  fa.d = d;
  fa.C = L.Cpad;
  fa.m_host = m;
  fa.id0_host = 0;
  fa.first = 1;
  fa.packed = L.packed;
  fa.shards = shards;
  KMPAR_HIP(timed_fold(ctx, kSlotDirect, dtype, DP, fa, s));
  KMPAR_HIP(launch_unpack_min(L.packed, (int)n, assign, D2, s));
  if (phi) KMPAR_HIP(launch_phi(D2, (int)n, L.phi_part, phi, s));
  return KMPAR_OK;
}

int kmpar_lloyd_until_stable(kmpar_ctx* ctx, const void* X, const float* row_scale,
                             kmpar_dtype dtype, int64_t n, int32_t d, float* C, int32_t k,
                             int32_t max_iters, int32_t* iters, int32_t* assign, double* phi,
                             void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  if (max_iters < 0) return set_err(ctx, KMPAR_E_INVAL, "max_iters=%d < 0", max_iters);
  if (!iters) return set_err(ctx, KMPAR_E_INVAL, "iters is NULL");
  if (assign && !aligned16(assign)) return set_err(ctx, KMPAR_E_INVAL, "assign misaligned");
  if (phi && ((uintptr_t)phi & 7u)) return set_err(ctx, KMPAR_E_INVAL, "phi misaligned");
  if (k > n) return set_err(ctx, KMPAR_E_INVAL, "k=%d > n", k);
  AssignLayout L;
  FoldArgs fa;
  int rc = assign_common(ctx, KMPAR_OP_LLOYD, X, row_scale, dtype, n, d, C, k, ws, ws_bytes, &L, &fa);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  int* cur = L.A;
  int* prev = L.A2;
  *iters = max_iters;
  for (int it = 0; it <= max_iters; ++it) {
    FoldArgs fi = fa;
    fi.A = cur;
    KMPAR_HIP(launch_pad_rows(C, k, d, padded_dim(d), L.Cpad, s));
    if ((rc = assign_pass(ctx, dtype, L, fi, k, s, it > 0))) return rc;
    if (phi) KMPAR_HIP(launch_phi(L.D2, (int)n, L.phi_part, phi + it, s));
    if (it > 0) {
      // one host read per iteration: the call cannot be captured in a graph
      KMPAR_HIP(launch_count_changed(cur, prev, (int)n, L.changed, s));
      int changed = -1;
      KMPAR_HIP(hipMemcpyAsync(&changed, L.changed, sizeof(int), hipMemcpyDeviceToHost, s));
      KMPAR_HIP(hipStreamSynchronize(s));
      if (changed == 0) {
        *iters = it;
        break;
      }
    }
    if (it == max_iters) break;
    KMPAR_HIP(launch_lloyd_update(dtype, X, row_scale, (int)n, d, cur, k, C, L.lw, s));
    int* t = cur;
    cur = prev;
    prev = t;
  }
  if (assign) KMPAR_HIP(launch_copy_i32(cur, assign, n, s));
  return KMPAR_OK;
}

int kmpar_workspace_size_batched(const kmpar_ctx* cctx, const kmpar_instance* inst_host,
                                 int32_t count, kmpar_dtype dtype, size_t* bytes_out) {
  kmpar_ctx* ctx = const_cast<kmpar_ctx*>(cctx);
  if (!bytes_out || !inst_host || count < 1) return set_err(ctx, KMPAR_E_INVAL, "bad batch arguments");
  if (dtype != KMPAR_F32 && dtype != KMPAR_BF16 && dtype != KMPAR_FP8_E4M3)
    return set_err(ctx, KMPAR_E_INVAL, "unknown dtype");
  const int rounds = inst_host[0].rounds;
  for (int i = 0; i < count; ++i) {
    const kmpar_instance& I = inst_host[i];
    if (I.n < 1 || I.n >= (int64_t)1 << 31 || I.d < 1 || I.d > kMaxD || I.k < 1 || I.k > I.n ||
        I.k > kMaxK || !ell_ok(I.ell) || I.rounds != rounds || rounds < 0 ||
        rounds > KMPAR_MAX_ROUNDS)
      return set_err(ctx, KMPAR_E_INVAL, "instance %d out of range", i);
  }
  int G = 0, dps[kBatchMaxGroups];
  *bytes_out = batched_workspace(inst_host, count, rounds, &G, dps);
  return KMPAR_OK;
}

int kmpar_init_batched(kmpar_ctx* ctx, const kmpar_instance* inst_host,
                       const kmpar_instance* inst_dev, int32_t count, kmpar_dtype dtype,
                       uint64_t seed, void* ws, size_t ws_bytes, const kmpar_trace* traces_dev,
                       void* stream) {
  if (!ctx) return KMPAR_E_INVAL;
  if (!inst_dev || !aligned16(inst_dev)) return set_err(ctx, KMPAR_E_INVAL, "inst_dev NULL/misaligned");
  size_t need = 0;
  int rc = kmpar_workspace_size_batched(ctx, inst_host, count, dtype, &need);
  if (rc) return rc;
  for (int i = 0; i < count; ++i) {
    const kmpar_instance& I = inst_host[i];
    if ((rc = check_common(ctx, I.X, I.row_scale, dtype, I.n, I.d))) return rc;
    if (!I.centers || !aligned16(I.centers))
      return set_err(ctx, KMPAR_E_INVAL, "instance %d: centers NULL/misaligned", i);
    if (I.stats && ((uintptr_t)I.stats & 7u))
      return set_err(ctx, KMPAR_E_INVAL, "instance %d: stats misaligned", i);
  }
  if (!ws) return set_err(ctx, KMPAR_E_INVAL, "workspace is NULL");
  if (ws_bytes < need)
    return set_err(ctx, KMPAR_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
  if ((rc = device_ready(ctx))) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return hip_fail(ctx, g.e, "hipSetDevice");
  if (traces_dev && ((uintptr_t)traces_dev & 7u))
    return set_err(ctx, KMPAR_E_INVAL, "traces_dev misaligned");
  hipStream_t s = (hipStream_t)stream;
  const LaunchTimer fold_timer = [&](const std::function<hipError_t()>& launch) {
    return timed(ctx, kSlotBatchFold, 0, nullptr, nullptr, 0, s, launch);
  };
  KMPAR_HIP(launch_batched(dtype, inst_host, inst_dev, count, inst_host[0].rounds, seed, ws,
                           traces_dev, &ctx->tuner, ctx->prof ? &fold_timer : nullptr, s));
  return KMPAR_OK;
}

}  // extern "C"
