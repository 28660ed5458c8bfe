// Host-side address checker of the library's kernels.
//
// For chosen blocks of each launch it replays, thread by thread, the index
// arithmetic of
//   * the REFINED screen (screen_body in screen_mfma.hip): candidate chunk
//     staging, biases, A operands (prepared or read from X), row scales,
//     the MFMA operand and bias reads, the per-wave merge, the staging of
//     the wave's rows, the refinement reads, D2 / A / S and the list;
//   * the operand preparation (k_prep_a, k_first_prep, k_prep_b);
//   * the few-center folds (k_fold_stream, k_fold_few) and the k-means++ step
//     and its first-level pick reduction;
//   * the listed-point rescan (k_rescan, k_rescan_merge);
//   * the Lloyd update (k_sort_count, k_sort_scatter, k_chunk_list,
//     k_seg_sum, k_centroid), run on a concrete assignment;
// and checks every global and LDS access against the extent of the buffer it
// addresses, with buffer sizes taken from the same geometry functions the
// workspace layouts use (geometry.hpp).  Data-dependent indices take every
// value the kernel can produce (the screen winner j1 anywhere in the pass's
// tiles; listed points anywhere in [0, n)).  The Lloyd update is simulated on
// an assignment with points that have no valid center, and every sorted
// position a centroid slice reads must have been written by the scatter.
//
// Shapes: the benchmark shapes (n = 4.8M x 42 FP32, 16M x 128 BF16, 50M x
// 256 FP8), every k-step count of the screen, ragged small shapes, and the
// shapes of three screen variants that stopped with memory faults and were
// taken out of the library (FP8 rows against two-term FP32 centers at
// 50M x 256, k = 2000; FP32 rows at d = 128; the batched groups d = 32, 64,
// 128) at which the shared screen code still runs its arithmetic.
//
// Usage: addr_check [--legacy-chunk-end]
//   --legacy-chunk-end  model the earlier chunk list, whose last cluster ran
//                       to n (the checker must then report the reads of
//                       unwritten sorted positions).
// Exit status 0 when no access leaves its buffer; 1 otherwise.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1203_6402_amd/csrc/geometry.hpp"

using namespace kmpar;

namespace {

enum Dtype { F32 = 0, BF16 = 1, FP8 = 2 };
int elem_size(Dtype t) { return t == F32 ? 4 : (t == BF16 ? 2 : 1); }
const char* dname(Dtype t) { return t == F32 ? "f32" : (t == BF16 ? "bf16" : "fp8"); }

struct Checker {
  long long checks = 0, bad = 0;
  std::string where;
  // [lo, lo + len) must lie in [0, size) (bytes).
  void in(const char* buf, int64_t lo, int64_t len, int64_t size, int64_t blk, int tid) {
    ++checks;
    if (lo >= 0 && len >= 0 && lo + len <= size) return;
    if (++bad <= 20)
      std::printf("  OUT OF BOUNDS %s: %s bytes [%lld, %lld) of %lld (block %lld, thread %d)\n",
                  where.c_str(), buf, (long long)lo, (long long)(lo + len), (long long)size,
                  (long long)blk, tid);
  }
  void fail(const std::string& msg) {
    ++bad;
    std::printf("  FAIL %s: %s\n", where.c_str(), msg.c_str());
  }
};

// Blocks to replay: the first and last few and a seeded sample between.
std::vector<int64_t> pick_blocks(int64_t nblocks, int sample, uint64_t seed) {
  std::vector<int64_t> b;
  for (int64_t i = 0; i < std::min<int64_t>(3, nblocks); ++i) b.push_back(i);
  for (int64_t i = std::max<int64_t>(0, nblocks - 3); i < nblocks; ++i) b.push_back(i);
  std::mt19937_64 r(seed);
  for (int i = 0; i < sample && nblocks > 6; ++i) b.push_back((int64_t)(r() % (uint64_t)nblocks));
  std::sort(b.begin(), b.end());
  b.erase(std::unique(b.begin(), b.end()), b.end());
  return b;
}

// ------------------------------------------------------------- the screen
struct ScreenShape {
  Dtype t;
  int split;      // 1, 2 or 3 bf16 terms
  int n, d;
  int m, id0;     // this pass: candidates [id0, id0 + m) of the row buffer
  int64_t crows;  // rows of the candidate row buffer (DP-padded FP32)
  int tiles_cap;  // B / ncg / scg capacity in tiles of 16
  int max_tiles;  // k_prep_b grid
  bool direct;    // A operands read from X (no prepared copy)
  bool first;
  bool codes;     // FP8 rows against rows of X: B operands are codes of X rows
  int64_t xrows;  // rows of X that candidate ids may name (codes)
};

// k_prep_b: one wave per tile of 16 candidates.
void check_prep_b(Checker& ck, const ScreenShape& s) {
  const int KS = screen_ksteps(s.split, s.d), DP = padded_dim_hd(s.d);
  const int64_t Bsz = (int64_t)screen_b_bytes(s.tiles_cap, s.d);
  const int64_t Csz = s.crows * DP * 4, Xsz = s.xrows * s.d, cand_sz = s.crows * 4;
  for (int q = 0; q < s.max_tiles; ++q) {
    if (q * 16 >= s.m) break;
    for (int lane = 0; lane < 64; ++lane) {
      const int j = q * 16 + lane % 16;
      const bool valid = j < s.m;
      // init rounds read the candidate at position j through cperm: any of
      // the pass's candidates; the last one stands for them here
      if (!s.first && valid) ck.in("cperm", (int64_t)j * 4, 4, (int64_t)s.tiles_cap * 16 * 4, q, lane);
      const int src = valid ? (s.first ? j : s.m - 1) : 0;
      const int64_t crow = (int64_t)(s.id0 + src) * DP;
      if (s.codes && valid) ck.in("cand", (int64_t)(s.id0 + src) * 4, 4, cand_sz, q, lane);
      for (int st = 0; st < KS; ++st) {
        for (int e = 0; e < 8; ++e) {
          const int k = st * 32 + (lane / 16) * 8 + e;
          const int part = k / s.d, coord = k - part * s.d;
          if (valid && part < s.split) {
            if (s.codes)  // any row of X may be a candidate
              ck.in("X codes", (s.xrows - 1) * (int64_t)s.d + coord, 1, Xsz, q, lane);
            else
              ck.in("C", (crow + coord) * 4, 4, Csz, q, lane);
          }
        }
        ck.in("B", (((int64_t)q * KS + st) * 64 + lane) * 16, 16, Bsz, q, lane);
      }
      if (lane < 16) {
        if (valid)
          for (int e = 0; e < s.d; e += std::max(1, s.d - 1)) ck.in("C norm", (crow + e) * 4, 4, Csz, q, lane);
        ck.in("ncg", (int64_t)j * 4, 4, (int64_t)s.tiles_cap * 16 * 4, q, lane);
        if (s.codes) {
          ck.in("scg", (int64_t)j * 4, 4, (int64_t)s.tiles_cap * 16 * 4, q, lane);
          if (valid) ck.in("row_scale", (s.xrows - 1) * 4, 4, s.xrows * 4, q, lane);
        }
      }
    }
  }
}

void check_screen(Checker& ck, const ScreenShape& s, int sample) {
  const bool SC = s.t == FP8;
  const int Sz = elem_size(s.t), d = s.d, DP = padded_dim_hd(d);
  const int KS = screen_ksteps(s.split, d);
  if (KS < 1 || KS > kScreenMaxKS) {
    ck.fail("k-steps out of range");
    return;
  }
  const int KRT = screen_krt(KS, SC), WP = KRT * 16, BP = kWaves * WP;
  // the single-group screen runs passes of at most kScreenOneGroupMaxTiles
  // tiles (the host's choice from the pass capacity)
  const bool oneg = s.max_tiles <= kScreenOneGroupMaxTiles;
  const int STAGE = screen_stage_bytes(KS, oneg, SC), WSTAGE = screen_wave_stage(KS, oneg, SC);
  const int CT = screen_chunk_tiles(KS, oneg, SC), CHUNK_V = CT * KS * 64;
  if (CT < 1 || CT * KS * 64 * 16 > STAGE) ck.fail("chunk exceeds its staging buffer");
  if (2 * STAGE != kWaves * WSTAGE) ck.fail("wave shares do not tile the staging buffers");
  const bool BCAST = screen_bcast(KS, oneg, SC);
  const int nW = BCAST ? 4 : (SC ? 2 : 1);
  const int64_t sBsz = 2LL * STAGE, sNsz = 2LL * CT * 16 * nW * 4;
  if (screen_three_waves(KS, oneg, SC) && 3 * (sBsz + sNsz) > 160 * 1024)
    ck.fail("three blocks of the three-wave screen exceed a CU's LDS");
  if (oneg && s.m > 0 && (s.m + 15) / 16 > (1 << screen_pass_tag_bits(s.max_tiles)))
    ck.fail("tile tags cannot number the pass");
  const int NBT = (CT * 16 + kWaves * 64 - 1) / (kWaves * 64);
  const int ntiles = (s.m + 15) / 16, nchunks = (ntiles + CT - 1) / CT;
  const int64_t n = s.n;
  const int64_t Xsz = n * d * Sz, Asz = (int64_t)screen_a_bytes(s.n, KS);
  const int64_t Bsz = (int64_t)screen_b_bytes(s.tiles_cap, d);
  const int64_t ncgsz = (int64_t)s.tiles_cap * 16 * 4, Csz = s.crows * DP * 4;
  if (ntiles > s.tiles_cap) ck.fail("pass has more tiles than the operand buffers");
  const int64_t nblocks = (n + BP - 1) / BP;
  for (int64_t blk : pick_blocks(nblocks, sample, (uint64_t)n * 131 + d)) {
    for (int tid = 0; tid < kWaves * 64; ++tid) {
      const int lane = tid % 64, wave = tid / 64;
      const int64_t wbase = blk * BP + (int64_t)wave * WP;
      // stage(c): direct loads of chunk c into buffer c & 1
      for (int c = 0; c < nchunks; ++c) {
        const int nt = std::min(CT, ntiles - c * CT), nv = nt * KS * 64;
        for (int v0 = wave * 64; v0 < nv; v0 += kWaves * 64) {
          ck.in("B chunk", ((int64_t)c * CHUNK_V + v0 + lane) * 16, 16, Bsz, blk, tid);
          ck.in("LDS sB", (int64_t)(c & 1) * STAGE + (int64_t)(v0 + lane) * 16, 16,
                (int64_t)(c & 1) * STAGE + STAGE, blk, tid);
        }
        // stage_ncg(c)
        for (int i = 0; i < NBT; ++i) {
          const int e = i * kWaves * 64 + tid;
          const int64_t idx = (int64_t)c * CT * 16 + e;
          if (e < CT * 16 && idx < (int64_t)ntiles * 16) {
            ck.in("ncg", idx * 4, 4, ncgsz, blk, tid);
            if (SC) ck.in("scg", idx * 4, 4, ncgsz, blk, tid);
          }
          // bias store of chunk c
          if (e < CT * 16) ck.in("LDS sN", ((int64_t)(c & 1) * CT * 16 * nW + (int64_t)e * nW) * 4, nW * 4, sNsz, blk, tid);
        }
        // operand and bias reads of the chunk's tiles
        for (int q = 0; q < nt; ++q) {
          for (int st = 0; st < KS; ++st)
            ck.in("LDS buf", (int64_t)(c & 1) * STAGE + ((int64_t)(q * KS + st) * 64 + lane) * 16, 16,
                  (int64_t)(c & 1) * STAGE + STAGE, blk, tid);
          ck.in("LDS ncs", ((int64_t)(c & 1) * CT * 16 * nW + (int64_t)(q * 16 + lane % 16) * nW) * 4,
                BCAST ? 16 : (SC ? 8 : 4), sNsz, blk, tid);
        }
      }
      // A operands
      for (int r = 0; r < KRT; ++r) {
        const int64_t tile = wbase / 16 + r;
        for (int st = 0; st < KS; ++st) {
          if (s.direct) {
            const int64_t p = wbase + r * 16 + lane % 16;
            const int k0 = st * 32 + (lane / 16) * 8;
            const int part = k0 / d, coord = k0 - part * d;
            if (p < n && part < s.split) {
              if (coord + 8 > d) ck.fail("direct A operand straddles a row (d % 8 != 0)");
              ck.in("X (A operand)", (p * d + coord) * Sz, 8 * Sz, Xsz, blk, tid);
            }
          } else {
            ck.in("Apre", ((tile * KS + st) * 64 + lane) * 16, 16, Asz, blk, tid);
          }
        }
        if (SC)
          for (int i = 0; i < 4; ++i) {
            const int64_t p = wbase + r * 16 + (lane / 16) * 4 + i;
            if (p < n) ck.in("row_scale", p * 4, 4, n * 4, blk, tid);
          }
      }
      // per-wave merge through the wave's share of sB, in halves when the
      // share cannot hold every point's entries
      const int64_t xw = (int64_t)wave * WSTAGE;
      const int HALVES = WP * 16 * 16 > WSTAGE ? 2 : 1, PH = WP / HALVES;
      for (int h = 0; h < HALVES; ++h) {
        for (int r = h * (KRT / HALVES); r < (h + 1) * (KRT / HALVES); ++r)
          for (int i = 0; i < 4; ++i) {
            const int pl = r * 16 + (lane / 16) * 4 + i - h * PH;
            ck.in("LDS M write", xw + (int64_t)(pl * 16 + ((lane % 16) ^ (pl & 15))) * 16, 16,
                  xw + WSTAGE, blk, tid);
          }
        if (lane / PH == h)
          for (int c = 0; c < 16; ++c)
            ck.in("LDS M read", xw + (int64_t)((lane - h * PH) * 16 + (c ^ (lane & 15))) * 16, 16,
                  xw + WSTAGE, blk, tid);
      }
      const int64_t p = wbase + lane;
      const bool valid = lane < WP && p < n;
      if (valid) {
        ck.in("norms", p * 4, 4, n * 4, blk, tid);
        if (!s.first) ck.in("D2", p * 4, 4, n * 4, blk, tid);
      }
      // staging of the wave's rows, groups of R
      const int64_t nvalid = std::max<int64_t>(0, std::min<int64_t>(WP, n - wbase));
      const int rowb = d * Sz;
      const int R = std::min(WP, (WSTAGE / rowb) & ~15);
      if (R < 16) ck.fail("staging group below 16 rows");
      const bool staged = nvalid == WP;
      // the winner j1: any column of the pass's tiles; refined only when j1 < m
      const int jmax_refined = s.m - 1;
      if (staged) {
        for (int c0 = 0; c0 < WP; c0 += R) {
          const int nr = std::min(R, WP - c0), bytes = nr * rowb;
          if (bytes % 16) ck.fail("staged group not whole 16-byte units");
          for (int v0 = 0; v0 < bytes; v0 += 1024)
            if (v0 + 16 * lane < bytes) {
              ck.in("X rows (staged)", (wbase + c0) * rowb + v0 + 16 * lane, 16, Xsz, blk, tid);
              ck.in("LDS rows", xw + v0 + 16 * lane, 16, xw + WSTAGE, blk, tid);
            }
          if (valid && lane >= c0 && lane < c0 + nr) {
            // refine_dist<XLDS>: 32 elements at a time from the staged row
            const int64_t xr = xw + (int64_t)(lane - c0) * rowb;
            const int64_t last = xr + (int64_t)((d + 31) / 32 * 32) * Sz;
            ck.in("LDS staged row", xr, last - xr, sBsz + sNsz, blk, tid);
          }
        }
      } else if (valid) {
        ck.in("X row (refine)", p * d * Sz, (int64_t)d * Sz, Xsz, blk, tid);
      }
      if (valid && s.m > 0 && !s.first)
        ck.in("cperm (winner)", (int64_t)jmax_refined * 4, 4, (int64_t)s.tiles_cap * 16 * 4, blk, tid);
      if (valid && s.m > 0) {
        for (int j1 : {0, jmax_refined}) {
          const int64_t row = (int64_t)(s.id0 + j1) * DP;
          for (int e0 = 0; e0 < d; e0 += 32)
            for (int u = 0; u < 8; ++u)
              if (e0 + 4 * u < d) {
                ck.in("C row (refine)", (row + e0 + 4 * u) * 4, 16, Csz, blk, tid);
                if (e0 + 4 * u + 4 > DP) ck.fail("float4 read past the padded row");
              }
        }
        ck.in("D2/A/S write", p * 4, 4, n * 4, blk, tid);
        ck.in("list", (n - 1) * 4, 4, n * 4, blk, tid);  // at most one entry per point
      }
    }
  }
}

// k_prep_a (PREP) / k_first_prep: blocks of 64 rows staged through LDS.
void check_prep_a(Checker& ck, Dtype t, int split, int n, int d, bool first, int64_t crows, int id0,
                  int sample) {
  const int KS = screen_ksteps(split, d), Sz = elem_size(t), EPV = 16 / Sz;
  const int pad = d % 32 == 0 ? 1 : 0, XS = d + pad, DP = padded_dim_hd(d);
  const int64_t lds = (int64_t)64 * XS * 4 + (first ? DP * 4 : 0);
  const int64_t Xsz = (int64_t)n * d * Sz, Asz = (int64_t)screen_a_bytes(n, KS);
  const int64_t nblocks = (int64_t)(n + kBlockPts - 1) / kBlockPts * (kBlockPts / 64);
  for (int64_t blk : pick_blocks(nblocks, sample, (uint64_t)n * 7 + d)) {
    const int64_t p0 = blk * 64;
    const int np = (int)std::max<int64_t>(0, std::min<int64_t>(64, n - p0));
    const int cnt = np * d, nvec = cnt * Sz / 16;
    for (int tid = 0; tid < 256; ++tid) {
      if (first)
        for (int e = tid; e < DP; e += 256) {
          ck.in("C first center", ((int64_t)id0 * DP + e) * 4, 4, crows * DP * 4, blk, tid);
          ck.in("LDS c0", ((int64_t)64 * XS + e) * 4, 4, lds, blk, tid);
        }
      if (t == FP8 && tid < np) ck.in("row_scale", (p0 + tid) * 4, 4, (int64_t)n * 4, blk, tid);
      for (int v0 = 0; v0 < nvec; v0 += 4 * 256)
        for (int u = 0; u < 4; ++u) {
          const int idx = v0 + u * 256 + tid;
          if (idx >= nvec) continue;
          ck.in("X rows", p0 * d * Sz + (int64_t)idx * 16, 16, Xsz, blk, tid);
          const int e = idx * EPV;
          int row = e / d, col = e - row * d;
          for (int k = 0; k < EPV; ++k) {
            ck.in("LDS xs", ((int64_t)e + k + row * pad) * 4, 4, (int64_t)64 * XS * 4, blk, tid);
            if (++col == d) {
              col = 0;
              ++row;
            }
          }
        }
      for (int e = nvec * EPV + tid; e < cnt; e += 256) {
        ck.in("X tail", (p0 * d + e) * Sz, Sz, Xsz, blk, tid);
        ck.in("LDS xs tail", ((int64_t)e + (e / d) * pad) * 4, 4, (int64_t)64 * XS * 4, blk, tid);
      }
      if (tid < np) {
        for (int e = 0; e < d; e += std::max(1, d - 1))
          ck.in("LDS row", ((int64_t)tid * XS + e) * 4, 4, (int64_t)64 * XS * 4, blk, tid);
        ck.in("norms/D2/A", (p0 + tid) * 4, 4, (int64_t)n * 4, blk, tid);
      }
      // write_a_operands
      const int lane = tid % 64, w = tid / 64, row = w * 16 + lane % 16;
      const bool valid = row < np;
      int part = 0, coord = (lane / 16) * 8;
      while (coord >= d) {
        coord -= d;
        ++part;
      }
      for (int st = 0; st < KS; ++st) {
        for (int e = 0; e < 8; ++e) {
          if (valid && part < split) {
            ck.in("LDS xs (operand)", ((int64_t)row * XS + coord) * 4, 4, (int64_t)64 * XS * 4, blk, tid);
            if (t == FP8) ck.in("X codes", (p0 + row) * d + coord, 1, Xsz, blk, tid);
          }
          if (++coord == d) {
            coord = 0;
            ++part;
          }
        }
        if (st + 1 < KS) {
          coord += 24;
          while (coord >= d) {
            coord -= d;
            ++part;
          }
        }
        ck.in("Apre", (((p0 / 16 + w) * KS + st) * 64 + lane) * 16, 16, Asz, blk, tid);
      }
    }
  }
}

// k_fold_stream: one wave of 64 points per block; full spans copied into
// LDS by 16-byte direct loads, the partial wave lane by lane.
void check_fold_stream(Checker& ck, Dtype t, int n, int d, int m, int id0, int64_t crows, int sample) {
  const int DP = padded_dim_hd(d), Sz = elem_size(t), rowb = d * Sz;
  const int64_t lds = (int64_t)64 * DP * Sz, Xsz = (int64_t)n * d * Sz, Csz = crows * DP * 4;
  if (DP > 64 || m > kStreamMaxM) ck.fail("stream fold outside its shape");
  if ((64 * rowb) % 16) ck.fail("span not whole 16-byte units");
  const int64_t nblocks = (n + 63) / 64;
  for (int64_t blk : pick_blocks(nblocks, sample, (uint64_t)n * 11 + d + m)) {
    const int64_t p0 = blk * 64;
    const bool full = p0 + 64 <= n;
    for (int lane = 0; lane < 64; ++lane) {
      const int64_t p = p0 + lane;
      const bool live = p < n;
      if (full) {
        for (int v0 = 0; v0 < 64 * rowb; v0 += 1024)
          if (v0 + 16 * lane < 64 * rowb) {
            ck.in("X span", p0 * rowb + v0 + 16 * lane, 16, Xsz, blk, lane);
            ck.in("LDS rows", v0 + 16 * lane, 16, lds, blk, lane);
          }
      } else if (live) {
        for (int j = 0; j < d; j += std::max(1, d - 1)) {
          ck.in("X row", (p * d + j) * Sz, Sz, Xsz, blk, lane);
          ck.in("LDS row copy", ((int64_t)lane * d + j) * Sz, Sz, lds, blk, lane);
        }
      }
      if (!live) continue;
      if (t == FP8) ck.in("row_scale", p * 4, 4, (int64_t)n * 4, blk, lane);
      ck.in("LDS row read", (int64_t)lane * rowb, rowb, lds, blk, lane);
      for (int c = 0; c < m; ++c) ck.in("C row", ((int64_t)(id0 + c) * DP) * 4, (int64_t)DP * 4, Csz, blk, lane);
      ck.in("D2/A", p * 4, 4, (int64_t)n * 4, blk, lane);
    }
  }
}

// k_kpp_step (k-means++ on all of X): one wave of 64 rows per block copied
// into a dynamic LDS buffer of 64 d elements, the latest center read per
// coordinate, D^2 read and written, one (key, index, sum) per block.
void check_kpp_step(Checker& ck, Dtype t, int n, int d, int sample) {
  const int Sz = elem_size(t), rowb = d * Sz;
  const int64_t lds = (int64_t)64 * d * Sz, Xsz = (int64_t)n * d * Sz;
  const int64_t nblocks = (n + 63) / 64;
  if ((64 * rowb) % 16) ck.fail("span not whole 16-byte units");
  for (int64_t blk : pick_blocks(nblocks, sample, (uint64_t)n * 13 + d)) {
    const int64_t p0 = blk * 64;
    for (int lane = 0; lane < 64; ++lane) {
      const int64_t i = p0 + lane;
      if (p0 + 64 <= n) {
        for (int v0 = 0; v0 < 64 * rowb; v0 += 1024)
          if (v0 + 16 * lane < 64 * rowb) {
            ck.in("X span", p0 * rowb + v0 + 16 * lane, 16, Xsz, blk, lane);
            ck.in("LDS rows", v0 + 16 * lane, 16, lds, blk, lane);
          }
      } else if (i < n) {
        ck.in("X row", i * d * Sz, (int64_t)d * Sz, Xsz, blk, lane);
        ck.in("LDS row copy", (int64_t)lane * d * Sz, (int64_t)d * Sz, lds, blk, lane);
      }
      if (i < n) {
        ck.in("LDS row read", (int64_t)lane * rowb, rowb, lds, blk, lane);
        ck.in("crow", 0, (int64_t)d * 4, (int64_t)d * 4, blk, lane);
        ck.in("D2", i * 4, 4, (int64_t)n * 4, blk, lane);
        if (t == FP8) ck.in("row_scale", i * 4, 4, (int64_t)n * 4, blk, lane);
      }
    }
    ck.in("block partials", blk * 8, 8, nblocks * 8, blk, 0);
  }
  // k_kpp_reduce: block q reads a run of the block partials, writes slot q
  const int64_t per = (nblocks + kKppQ - 1) / kKppQ;
  for (int q = 0; q < kKppQ; ++q) {
    const int64_t b0 = std::min(nblocks, q * per), b1 = std::min(nblocks, b0 + per);
    for (int tid = 0; tid < 256; ++tid)
      for (int64_t b = b0 + tid; b < b1; b += 256)
        ck.in("partials (reduce)", b * 8, 8, nblocks * 8, q, tid);
    ck.in("first-level slot", (int64_t)q * 8, 8, (int64_t)kKppQ * 8, q, 0);
  }
}

// k_fold_few: 64 rows staged through LDS per block of 256 threads, the
// four waves splitting up to kStagedMaxM candidates.
void check_fold_few(Checker& ck, Dtype t, int n, int d, int m, int id0, int64_t crows, int sample) {
  const int DP = padded_dim_hd(d), Sz = elem_size(t), EPV = 16 / Sz;
  const int pad = d % 32 == 0 ? 1 : 0, XS = d + pad;
  const int64_t xs_sz = (int64_t)64 * (DP + 1) * 4, Xsz = (int64_t)n * d * Sz, Csz = crows * DP * 4;
  if (DP > 64 || m > kStagedMaxM) ck.fail("few-center fold outside its shape");
  const int64_t nblocks = (n + 63) / 64;
  for (int64_t blk : pick_blocks(nblocks, sample, (uint64_t)n * 5 + d + m)) {
    const int64_t p0 = blk * 64;
    const int np = (int)std::max<int64_t>(0, std::min<int64_t>(64, n - p0));
    const int cnt = np * d, nvec = cnt * Sz / 16;
    for (int tid = 0; tid < 256; ++tid) {
      if (t == FP8 && tid < np) ck.in("row_scale", (p0 + tid) * 4, 4, (int64_t)n * 4, blk, tid);
      for (int v0 = 0; v0 < nvec; v0 += 4 * 256)
        for (int u = 0; u < 4; ++u) {
          const int idx = v0 + u * 256 + tid;
          if (idx >= nvec) continue;
          ck.in("X rows", p0 * d * Sz + (int64_t)idx * 16, 16, Xsz, blk, tid);
          const int e = idx * EPV;
          int row = e / d, col = e - row * d;
          for (int k = 0; k < EPV; ++k) {
            ck.in("LDS xs", ((int64_t)e + k + row * pad) * 4, 4, xs_sz, blk, tid);
            if (++col == d) {
              col = 0;
              ++row;
            }
          }
        }
      for (int e = nvec * EPV + tid; e < cnt; e += 256) {
        ck.in("X tail", (p0 * d + e) * Sz, Sz, Xsz, blk, tid);
        ck.in("LDS xs tail", ((int64_t)e + (e / d) * pad) * 4, 4, xs_sz, blk, tid);
      }
      const int w = tid / 64, pl = tid % 64;
      for (int j = 0; j < d; j += std::max(1, d - 1))
        if (pl < np) ck.in("LDS row", ((int64_t)pl * XS + j) * 4, 4, xs_sz, blk, tid);
      for (int c = w; c < m; c += 4)
        ck.in("C row", ((int64_t)(id0 + c) * DP) * 4, (int64_t)DP * 4, Csz, blk, tid);
      if (w == 0 && pl < np) ck.in("D2/A", (p0 + pl) * 4, 4, (int64_t)n * 4, blk, tid);
    }
  }
}

// k_cand_sort: one block of 1024 threads over the m candidates of a pass
// (keys, bucket counts, positions from the bucket offsets, tile intervals).
void check_cand_sort(Checker& ck, int m, int d, int id0, int64_t crows, int tiles_cap) {
  const int DP = padded_dim_hd(d);
  const int64_t Csz = crows * DP * 4, cap16 = (int64_t)tiles_cap * 16;
  const int ntiles = (m + 15) / 16;
  if (ntiles > tiles_cap) ck.fail("sort: pass has more tiles than cperm / tnr");
  if (kCandBuckets != 1024) ck.fail("sort: one bucket per thread");
  for (int tid = 0; tid < 1024; ++tid) {
    if (m > kCandSortMax) {
      for (int pos = tid; pos < ntiles * 16; pos += 1024) ck.in("cperm", (int64_t)pos * 4, 4, cap16 * 4, 0, tid);
      for (int q = tid; q < ntiles; q += 1024) ck.in("tnr", (int64_t)q * 8, 8, (int64_t)tiles_cap * 8, 0, tid);
      continue;
    }
    ck.in("LDS bucket", (int64_t)tid * 4, 4, (int64_t)kCandBuckets * 4, 0, tid);
    for (int i = tid; i < m; i += 1024) {
      ck.in("C row (sort)", ((int64_t)(id0 + i) * DP) * 4, (int64_t)d * 4, Csz, 0, tid);
      ck.in("LDS key", (int64_t)i * 4, 4, (int64_t)kCandSortMax * 4, 0, tid);
      // positions are bucket offsets plus arrivals: some pos in [0, m)
      ck.in("cperm (pos)", (int64_t)(m - 1) * 4, 4, cap16 * 4, 0, tid);
      ck.in("LDS skey (pos)", (int64_t)(m - 1) * 4, 4, (int64_t)kCandSortMax * 4, 0, tid);
    }
    for (int pos = m + tid; pos < ntiles * 16; pos += 1024) ck.in("cperm (pad)", (int64_t)pos * 4, 4, cap16 * 4, 0, tid);
    for (int q = tid; q < ntiles; q += 1024) {
      for (int pos = q * 16; pos < std::min(m, q * 16 + 16); ++pos)
        ck.in("LDS skey (tile)", (int64_t)pos * 4, 4, (int64_t)kCandSortMax * 4, 0, tid);
      ck.in("tnr", (int64_t)q * 8, 8, (int64_t)tiles_cap * 8, 0, tid);
    }
  }
}

// k_rescan + k_rescan_merge for a list of nlist points.
void check_rescan(Checker& ck, Dtype t, int n, int d, int m, int id0, int64_t crows, int nlist) {
  const int DP = padded_dim_hd(d), Sz = elem_size(t);
  const int P = kRescanPts, CC = kRescanCands, NS = 256 / P, NV = (CC * (DP / 4) + 255) / 256;
  const int XS = DP + 1, CSTR = DP + 4;
  int grid = (n + P - 1) / P;
  grid = std::min(grid, kRescanMaxItems);
  const int groups = (nlist + P - 1) / P;
  int S = 1;
  while (S < kRescanMaxSplit && groups * S * 2 <= grid) S *= 2;
  const int nch = (m + CC - 1) / CC;
  const int64_t Csz = crows * DP * 4, Xsz = (int64_t)n * d * Sz;
  const int64_t rpart_sz = (int64_t)kRescanMaxItems * kRescanPts * 16;
  const int64_t lds_xs = (int64_t)P * XS * 4, lds_cs = (int64_t)CC * CSTR * 4;
  std::vector<int64_t> items = pick_blocks((int64_t)groups * S, 24, (uint64_t)nlist * 3 + d);
  for (int64_t it : items) {
    const int g = (int)(it / S), sl = (int)(it - (int64_t)g * S);
    const int np = std::min(P, nlist - g * P);
    const int cbeg = (sl * nch / S) * CC, cend = std::min(m, ((sl + 1) * nch / S) * CC);
    for (int tid = 0; tid < 256; ++tid) {
      const int r = tid % P, slot = tid / P;
      for (int idx = tid; idx < P * DP; idx += 256) {
        const int q = idx / DP, e = idx - q * DP;
        if (q < np && e < d) {
          ck.in("list", ((int64_t)g * P + q) * 4, 4, (int64_t)n * 4, it, tid);
          ck.in("X listed row", ((int64_t)(n - 1) * d + e) * Sz, Sz, Xsz, it, tid);
        }
        ck.in("LDS xs", ((int64_t)q * XS + e) * 4, 4, lds_xs, it, tid);
      }
      for (int c0 = cbeg; c0 < cend; c0 += CC) {
        const int nc = std::min(CC, cend - c0);
        for (int u = 0; u < NV; ++u) {
          const int idx = tid + u * 256;
          const int j = idx / (DP / 4), e4 = idx - j * (DP / 4);
          if (idx < CC * (DP / 4) && j < nc)
            ck.in("C chunk", ((int64_t)(id0 + c0 + j) * DP + e4 * 4) * 4, 16, Csz, it, tid);
          if (idx < CC * (DP / 4)) ck.in("LDS cs", ((int64_t)j * CSTR + e4 * 4) * 4, 16, lds_cs, it, tid);
        }
        for (int e = 0; e < DP; e += 4) {
          ck.in("LDS xr", ((int64_t)r * XS + e) * 4, 16, lds_xs, it, tid);
          for (int i = 0; i < CC / NS; ++i)
            ck.in("LDS cv", ((int64_t)(slot + NS * i) * CSTR + e) * 4, 16, lds_cs, it, tid);
        }
      }
      if (slot == 0 && r < np) {
        if (S == 1) ck.in("list/D2", ((int64_t)g * P + r) * 4, 4, (int64_t)n * 4, it, tid);
        else ck.in("rpart", (it * P + r) * 16, 16, rpart_sz, it, tid);
      }
    }
  }
  if (S > 1)  // k_rescan_merge
    for (int i = 0; i < nlist; ++i) {
      const int g = i / P, r = i - g * P;
      for (int sl = 0; sl < S; ++sl) ck.in("rpart (merge)", (((int64_t)g * S + sl) * P + r) * 16, 16, rpart_sz, i, 0);
    }
}

// ---------------------------------------------------------- Lloyd update
// Simulates the counting sort on a concrete assignment and checks the
// centroid sums' reads.
void check_lloyd(Checker& ck, Dtype t, int n, int d, int k, const std::vector<int>& A, bool legacy) {
  const int nbs = (n + kSortChunk - 1) / kSortChunk;
  const int64_t keys = legacy ? k : (int64_t)k + 1;
  const int64_t L = keys * nbs;
  const int64_t bcnt_sz = ((int64_t)k + 1) * nbs;  // the workspace's table
  if (L > bcnt_sz) ck.fail("count table larger than its buffer");
  std::vector<int> bcnt(L, 0);
  auto key_of = [&](int a) { return (a >= 0 && a < k) ? a : (legacy ? -1 : k); };
  for (int b = 0; b < nbs; ++b)
    for (int i = b * kSortChunk; i < std::min(n, (b + 1) * kSortChunk); ++i) {
      const int key = key_of(A[i]);
      if (key >= 0) ++bcnt[(int64_t)key * nbs + b];
    }
  // exclusive scan (k_scan_*)
  int64_t run = 0;
  for (int64_t j = 0; j < L; ++j) {
    const int v = bcnt[j];
    bcnt[j] = (int)run;
    run += v;
  }
  // scatter: every point with a key gets its slot
  std::vector<int> sorted(n, -1);
  std::vector<char> written(n, 0);
  for (int b = 0; b < nbs; ++b) {
    std::vector<int64_t> cur(keys);
    for (int64_t c = 0; c < keys; ++c) cur[c] = bcnt[c * nbs + b];
    for (int i = b * kSortChunk; i < std::min(n, (b + 1) * kSortChunk); ++i) {
      const int key = key_of(A[i]);
      if (key < 0) continue;
      const int64_t pos = cur[key]++;
      ck.in("sorted (scatter)", pos * 4, 4, (int64_t)n * 4, b, 0);
      if (pos >= 0 && pos < n) {
        sorted[pos] = i;
        written[pos] = 1;
      }
    }
  }
  // chunk list
  std::vector<int> coff(k + 1), cstart(k + 1);
  int64_t chunks = 0;
  for (int c = 0; c < k; ++c) {
    const int o = bcnt[(int64_t)c * nbs];
    const int o1 = legacy ? ((c + 1 < k) ? bcnt[(int64_t)(c + 1) * nbs] : n) : bcnt[(int64_t)(c + 1) * nbs];
    coff[c] = o;
    cstart[c] = (int)chunks;
    chunks += (o1 - o + kSegChunk - 1) / kSegChunk;
  }
  coff[k] = legacy ? n : bcnt[(int64_t)k * nbs];
  cstart[k] = (int)chunks;
  const int64_t max_chunks = (n + kSegChunk - 1) / kSegChunk + k;
  if (chunks > max_chunks) ck.fail("more chunks than the segment-sum grid");
  const int64_t part_sz = max_chunks * d * 8;
  const int64_t Xsz = (int64_t)n * d * elem_size(t);
  const int DW = seg_width(d), NSL = 256 / DW;
  int64_t unwritten = 0;
  for (int64_t q = 0; q < chunks; ++q) {
    int lo = 0, hi = k;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (cstart[mid] <= q) lo = mid; else hi = mid;
    }
    const int c = lo;
    const int p0 = coff[c] + (int)(q - cstart[c]) * kSegChunk;
    const int p1 = std::min(coff[c + 1], p0 + kSegChunk);
    for (int sl = 0; sl < NSL; ++sl) {
      const int len = p1 - p0, per = (len + NSL - 1) / NSL;
      const int a = p0 + std::min(len, sl * per), b = p0 + std::min(len, (sl + 1) * per);
      for (int p = a; p < b; ++p) {
        ck.in("sorted (sum)", (int64_t)p * 4, 4, (int64_t)n * 4, q, sl);
        if (p >= 0 && p < n && !written[p]) ++unwritten;
        else if (p >= 0 && p < n)
          ck.in("X (sum)", ((int64_t)sorted[p] * d + d - 1) * elem_size(t), elem_size(t), Xsz, q, sl);
      }
    }
    ck.in("part", (q * d + d - 1) * 8, 8, part_sz, q, 0);
  }
  if (unwritten) ck.fail(std::to_string(unwritten) + " sorted positions read before any scatter wrote them");
  for (int c = 0; c < k; ++c)
    for (int q = cstart[c]; q < cstart[c + 1]; ++q) ck.in("part (centroid)", ((int64_t)q * d) * 8, 8, part_sz, c, 0);
}

}  // namespace

int main(int argc, char** argv) {
  bool legacy = argc > 1 && std::strcmp(argv[1], "--legacy-chunk-end") == 0;
  Checker ck;
  auto run = [&](const std::string& what, auto fn) {
    ck.where = what;
    const long long b0 = ck.bad;
    fn();
    std::printf("%-78s %s\n", what.c_str(), ck.bad == b0 ? "ok" : "VIOLATIONS");
  };

  if (!legacy) {
    // ---- the screen at init passes (centers are rows of X)
    struct InitCase { const char* name; Dtype t; int n, d; double ell; int rounds; };
    std::vector<InitCase> inits = {
        {"C1 4.8M x 42 f32 ell=1000", F32, 4800000, 42, 1000.0, 5},
        {"C1 4.8M x 42 f32 ell=250", F32, 4800000, 42, 250.0, 5},
        {"C2 16M x 128 bf16 ell=2000", BF16, 16000000, 128, 2000.0, 5},
        {"C3 50M x 256 fp8 ell=4000", FP8, 50000000, 256, 4000.0, 5},
        {"ragged 10001 x 15 f32", F32, 10001, 15, 100.0, 5},
        {"ragged 5003 x 85 f32 (K=256)", F32, 5003, 85, 80.0, 4},
        {"ragged 4001 x 128 f32 (two row tiles)", F32, 4001, 128, 60.0, 3},
        {"ragged 2503 x 170 f32 (K=512)", F32, 2503, 170, 50.0, 3},
        {"1M+7 x 100 f32 (two row tiles)", F32, 1000007, 100, 2000.0, 5},
        {"ragged 777 x 250 bf16", BF16, 777, 250, 64.0, 3},
        {"ragged 3001 x 37 bf16 (prepared A)", BF16, 3001, 37, 80.0, 4},
        {"ragged 2049 x 200 fp8 (two row tiles)", FP8, 2049, 200, 64.0, 4},
        {"ragged 999 x 24 fp8", FP8, 999, 24, 40.0, 4},
    };
    for (int d = 1; d <= 170; d += 13)
      inits.push_back({"sweep f32", F32, 3000 + d, d, 50.0, 3});
    for (const auto& c : inits) {
      const int split = c.t == F32 ? 3 : 1;
      const int64_t cap = cap_round_hd(c.n, c.ell);
      const int64_t capT = 1 + (int64_t)c.rounds * cap;
      const int tiles = (int)((cap + 15) / 16);
      const bool direct = (c.t == BF16 && c.d % 8 == 0) || (c.t == FP8 && c.d % 8 == 0);
      if (screen_ksteps(split, c.d) > kScreenMaxKS) continue;
      const std::string tag = std::string(c.name) + " [" + dname(c.t) + " d=" + std::to_string(c.d) + "]";
      for (int64_t m : {(int64_t)1, (int64_t)15, (int64_t)16, (int64_t)17, cap - 1, cap}) {
        if (m < 1 || m > cap) continue;
        for (int64_t id0 : {(int64_t)1, capT - m}) {
          ScreenShape s{c.t, split, c.n, c.d, (int)m, (int)id0, capT, tiles, tiles, direct, false,
                        c.t == FP8, c.n};
          run("screen " + tag + " m=" + std::to_string(m) + " id0=" + std::to_string(id0),
              [&] { check_screen(ck, s, 12); });
          run("prep_b " + tag + " m=" + std::to_string(m), [&] { check_prep_b(ck, s); });
          run("cand_sort " + tag + " m=" + std::to_string(m),
              [&] { check_cand_sort(ck, (int)m, c.d, (int)id0, capT, tiles); });
        }
      }
      if (!direct)
        run("first_prep " + tag, [&] { check_prep_a(ck, c.t, split, c.n, c.d, true, capT, 0, 24); });
      for (int nl : {1, 31, 33, 5000, 16384, c.n})
        if (nl <= c.n)
          run("rescan " + tag + " list=" + std::to_string(nl),
              [&] { check_rescan(ck, c.t, c.n, c.d, (int)cap, (int)(capT - cap), capT, nl); });
    }
    // ---- assignment passes (FP32 centers: split 3 for FP32 rows, 2 for BF16)
    struct AsgCase { const char* name; Dtype t; int split; int n, d, k; };
    std::vector<AsgCase> asg = {
        {"Lloyd C1 4.8M x 42 f32 k=500", F32, 3, 4800000, 42, 500},
        {"assign 16M x 128 bf16 k=1000", BF16, 2, 16000000, 128, 1000},
        {"assign 1M+3 x 256 bf16 k=2000 (two row tiles)", BF16, 2, 1000003, 256, 2000},
        {"assign 100003 x 128 f32 k=77 (two row tiles)", F32, 3, 100003, 128, 77},
        // the removed variants' shapes, through the shared screen code
        {"removed FP8-vs-centers screen: 50M x 256 fp8 k=2000", FP8, 2, 50000000, 256, 2000},
        {"removed norm-pruned screen: 2M x 128 f32 k=1000", F32, 3, 2000000, 128, 1000},
        {"removed batched screen: 200000 x 32 f32 k=448", F32, 3, 200000, 32, 448},
        {"removed batched screen: 200000 x 64 f32 k=448", F32, 3, 200000, 64, 448},
        {"removed batched screen: 200000 x 128 f32 k=448", F32, 3, 200000, 128, 448},
        {"removed batched screen: 2000 x 128 f32 k=46", F32, 3, 2000, 128, 46},
    };
    for (const auto& c : asg) {
      const int tiles = (c.k + 15) / 16;
      const bool direct = c.t == BF16 && c.d % 8 == 0;
      const std::string tag = std::string(c.name);
      ScreenShape s{c.t, c.split, c.n, c.d, c.k, 0, c.k, tiles, tiles, direct, true, false, c.n};
      run("screen " + tag, [&] { check_screen(ck, s, 16); });
      run("prep_b " + tag, [&] { check_prep_b(ck, s); });
      if (!direct) run("prep_a " + tag, [&] { check_prep_a(ck, c.t, c.split, c.n, c.d, false, c.k, 0, 24); });
      for (int nl : {1, 9000, c.n})
        if (nl <= c.n)
          run("rescan " + tag + " list=" + std::to_string(nl),
              [&] { check_rescan(ck, c.t, c.n, c.d, c.k, 0, c.k, nl); });
    }
  }

  // ---- assignment passes against few centers (staged rows)
  if (!legacy) {
    struct FewCase { const char* name; Dtype t; int n, d, m; };
    std::vector<FewCase> few = {
        {"staged C1 4.8M x 42 f32 m=1", F32, 4800000, 42, 1},
        {"staged C1 4.8M x 42 f32 m=64", F32, 4800000, 42, 64},
        {"staged 10007 x 64 f32 m=33", F32, 10007, 64, 33},
        {"staged 10007 x 32 bf16 m=5", BF16, 10007, 32, 5},
        {"staged 10007 x 3 fp8 m=2", FP8, 10007, 3, 2},
        {"staged 999 x 61 fp8 m=64", FP8, 999, 61, 64},
        {"staged 1 x 1 f32 m=1", F32, 1, 1, 1},
        {"staged 10007 x 64 f32 m=4", F32, 10007, 64, 4},
        {"staged 129 x 17 fp8 m=3", FP8, 129, 17, 3},
        {"staged 4.8M+5 x 42 f32 m=5", F32, 4800005, 42, 5},
    };
    for (const auto& c : few) {
      if (c.m <= kStreamMaxM)
        run(c.name, [&] { check_fold_stream(ck, c.t, c.n, c.d, c.m, 0, c.m, 16); });
      else
        run(c.name, [&] { check_fold_few(ck, c.t, c.n, c.d, c.m, 0, c.m, 16); });
    }
  }

  // ---- k-means++ steps
  if (!legacy) {
    run("kpp step C1 4.8M x 42 f32", [&] { check_kpp_step(ck, F32, 4800000, 42, 16); });
    run("kpp step 50M x 256 fp8", [&] { check_kpp_step(ck, FP8, 50000000, 256, 16); });
    run("kpp step 1001 x 7 bf16", [&] { check_kpp_step(ck, BF16, 1001, 7, 16); });
    run("kpp step 63 x 3 fp8", [&] { check_kpp_step(ck, FP8, 63, 3, 16); });
  }

  // ---- the Lloyd update on concrete assignments
  struct LloydCase { const char* name; Dtype t; int n, d, k; int invalid_every; };
  std::vector<LloydCase> ll = {
      {"Lloyd C3 50M x 256 fp8 k=2000", FP8, 50000000, 256, 2000, 0},
      {"Lloyd C1 4.8M x 42 f32 k=500", F32, 4800000, 42, 500, 0},
      {"Lloyd 100003 x 7 f32 k=16384", F32, 100003, 7, 16384, 0},
      {"Lloyd 70001 x 33 bf16 k=300, every 97th point without a center", BF16, 70001, 33, 300, 97},
      {"Lloyd 4097 x 5 f32 k=3, every 5th point without a center", F32, 4097, 5, 3, 5},
  };
  for (const auto& c : ll) {
    if (legacy && c.invalid_every == 0) continue;
    std::vector<int> A(c.n);
    std::mt19937_64 r(c.n);
    // skewed cluster sizes (one large cluster, the rest spread), some empty
    for (int i = 0; i < c.n; ++i) {
      const uint64_t u = r();
      A[i] = (u % 3 == 0) ? 0 : (int)((u >> 8) % (uint64_t)std::max(1, c.k - c.k / 10));
      if (c.invalid_every && i % c.invalid_every == 0) A[i] = (i / c.invalid_every) % 2 ? -1 : c.k;
    }
    run(std::string(legacy ? "[legacy chunk end] " : "") + c.name,
        [&] { check_lloyd(ck, c.t, c.n, c.d, c.k, A, legacy); });
  }
  std::printf("%lld accesses checked, %lld violations\n", ck.checks, ck.bad);
  return ck.bad ? 1 : 0;
}
