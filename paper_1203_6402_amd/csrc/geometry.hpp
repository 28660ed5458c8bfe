// Launch and buffer geometry of the kernels: block shapes, chunk sizes and
// buffer extents as plain integer functions.  The kernels, the workspace
// layouts and the host-side address checker all take them from here, so
// this header holds no HIP types and compiles as ordinary C++.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __HIPCC__
#define KMPAR_HD __host__ __device__
#else
#define KMPAR_HD
#endif

namespace kmpar {

// Padded row length used for candidate / center rows (zeros past d).
KMPAR_HD inline int padded_dim_hd(int d) {
  if (d <= 64) return (d + 3) / 4 * 4;
  if (d <= 128) return (d + 15) / 16 * 16;
  return (d + 31) / 32 * 32;
}

// Integer square root (floor), identical on host and device.
KMPAR_HD inline int64_t isqrt64(int64_t v) {
  int64_t r = 0;
  for (int64_t b = (int64_t)1 << 31; b > 0; b >>= 1)
    if ((r + b) * (r + b) <= v) r += b;
  return r;
}

// Per-round candidate capacity min(n, L + 12 isqrt(L) + 76), L = ceil(ell):
// at least ell + 12 sqrt(ell) + 64, i.e. more than 12 standard deviations
// above the expected ell kept points (Section 3.3).  Integer arithmetic, so
// host planning and device kernels agree exactly.
KMPAR_HD inline int64_t cap_round_hd(int64_t n, double ell) {
  const double c = ceil(ell);
  if (!(c < 4.0e18)) return n;
  const int64_t L = (int64_t)c;
  const int64_t cap = L + 12 * isqrt64(L) + 76;
  return cap < n ? cap : n;
}

// Point tile of the direct-form distance pass and the other chunked passes.
constexpr int kFoldBlock = 256;
constexpr int kPhiChunk = 4096;    // points per block of the phi reduction
constexpr int kDrawChunk = 2048;   // points per block of the draw passes
constexpr int kSortChunk = 4096;   // points per block of the Lloyd counting sort
constexpr int kSegChunk = 2048;    // sorted points per block of the centroid sums
constexpr int kScanTile = 4096;    // elements per tile of the three-phase scan
constexpr int kSortAhead = 16;     // 64-point key tiles loaded ahead by the scatter
constexpr int kSegAhead = 16;      // rows whose loads a centroid slice issues ahead

// Lanes per slice row of the centroid sums: the power of two covering d, at
// most 64.
KMPAR_HD inline int seg_width(int d) {
  int w = 1;
  while (w < d && w < 64) w <<= 1;
  return w;
}

// Assignment passes against at most this many centers (rows of up to 64
// padded elements) stage X through LDS (bound by HBM): one-wave blocks with
// direct global-to-LDS copies up to kStreamMaxM centers (k_fold_stream),
// four-wave blocks splitting the centers beyond (k_fold_few).
constexpr int kStreamMaxM = 4;
constexpr int kStagedMaxM = 64;

// Candidates of a pass that the norm sort of the screen's tiles handles
// (one block, keys in LDS); larger passes keep id order.
constexpr int kCandSortMax = 8192;
constexpr int kCandBuckets = 1024;  // log2 ||c||^2 buckets of that sort (one per thread)

// Blocks of the first level of the k-means++ pick (each reduces a run of
// the step's one-wave block partials).
constexpr int kKppQ = 256;

// Rescan of listed points: points per block step, grid limit (and slice-
// winner slots / kRescanPts), candidate rows per LDS chunk, most slices.
constexpr int kRescanPts = 32;
constexpr int kRescanMaxItems = 1024;
constexpr int kRescanCands = 32;
constexpr int kRescanMaxSplit = 8;

// ------------------------------------------------------------ the screen
// Largest number of 32-wide k-steps of the screen's operands.
constexpr int kScreenMaxKS = 16;
constexpr int kWaves = 4;               // waves per screen block
constexpr int kStageBytes = 32 * 1024;  // LDS per candidate staging buffer
// The single-group screen (a pass of at most kScreenOneGroupMaxTiles tiles,
// each value tagged with its tile's index in the pass) keeps no per-group
// maxima, which frees the registers for three waves per SIMD at up to four
// k-steps of unscaled rows; there its staging buffers shrink so that three
// blocks share a CU.
constexpr int kScreenOneGroupMaxTiles = 128;
constexpr bool screen_three_waves(int KS, bool oneg, bool scaled) { return oneg && KS <= 4 && !scaled; }
constexpr int screen_stage_bytes(int KS, bool oneg, bool scaled = false) {
  return screen_three_waves(KS, oneg, scaled) ? 24 * 1024 : kStageBytes;
}
// LDS bytes each wave reuses after the pass (a quarter of the two buffers).
constexpr int screen_wave_stage(int KS, bool oneg, bool scaled = false) {
  return screen_stage_bytes(KS, oneg, scaled) * 2 / kWaves;
}
// 16-point row tiles per wave: four while the A operands of KS k-steps fit
// the registers beside the accumulators and running maxima, two beyond 8.
// Rows with scales spend more registers per value (row scales, the scaled
// epilogue): two row tiles from five k-steps on.
constexpr int screen_krt(int KS, bool scaled) {
  return scaled ? (KS <= 4 ? 4 : 2) : (KS <= 8 ? 4 : 2);
}
constexpr int kBlockPts = kWaves * 4 * 16;  // the largest block (256 points)
// Candidate tiles per LDS chunk for KS k-steps, chunks per tag group (groups
// of up to 64 tiles), and the tag bits that number a tile within its group.
// A larger group merges its running maxima less often; its tag, in the low
// mantissa bits, moves each value by up to 2^(TB - 23) of its magnitude.
constexpr int kScreenGroupTiles = 64;
constexpr int screen_chunk_tiles(int KS, bool oneg = false, bool scaled = false) {
  return screen_stage_bytes(KS, oneg, scaled) / (KS * 64 * 16);
}
constexpr int screen_group_chunks(int KS) {
  return screen_chunk_tiles(KS) >= kScreenGroupTiles ? 1 : kScreenGroupTiles / screen_chunk_tiles(KS);
}
constexpr int screen_tag_bits(int KS) {
  int b = 0;
  while ((1 << b) < screen_group_chunks(KS) * screen_chunk_tiles(KS)) ++b;
  return b;
}
// Whether the biases of a chunk are stored four times over (one LDS read
// then gives an accumulator's initial value): unscaled rows with chunks of
// up to 16 tiles, up to 8 in the three-wave screen (its LDS budget).
constexpr bool screen_bcast(int KS, bool oneg, bool scaled) {
  return !scaled && screen_chunk_tiles(KS, oneg, scaled) <= (screen_three_waves(KS, oneg, scaled) ? 8 : 16);
}
// Tag bits of the single-group screen for a pass of up to max_tiles tiles.
constexpr int screen_pass_tag_bits(int max_tiles) {
  int b = 1;
  while ((1 << b) < max_tiles) ++b;
  return b;
}
// K axis of a split-term operand: SPLIT copies of d, in 32-wide k-steps.
constexpr int screen_ksteps(int split, int d) { return split ? (split * d + 31) / 32 : 0; }
// Prepared A operands: every tile of 16 points of whole 256-point blocks.
inline size_t screen_a_bytes(int n, int KS) {
  const size_t tiles = (size_t)(n + kBlockPts - 1) / kBlockPts * (kBlockPts / 16);
  return tiles * KS * 64 * 16;
}
// B operands for up to `tiles` tiles of 16 candidates at the widest split.
inline size_t screen_b_bytes(int tiles, int d) {
  return (size_t)tiles * screen_ksteps(3, d) * 64 * 16;
}

}  // namespace kmpar
