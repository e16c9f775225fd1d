// Internal declarations shared by the library's HIP translation units.
// Nothing here is part of the public C ABI (include/anyseq_mi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "anyseq_mi.h"

namespace asmi {

// One DPP row (16 lanes) cooperates on one alignment: lane t owns K adjacent
// DP columns and, in wavefront step `it`, computes row it + 1 - t
// (the paper's section 3.1 mapping with p = 16 lanes).  A wave64 therefore
// carries four independent alignments.
constexpr int kGroup = 16;
constexpr int kWave = 64;
constexpr int kGroupsPerWave = kWave / kGroup;

// Finite stand-in for -infinity in 32-bit cells.  Every reachable value stays
// far above it (scores are bounded a priori, see RangeBound in runtime.hip).
constexpr int32_t kNegInf32 = -(1 << 29);

enum Mode : int32_t { kGlobal = 0, kSemiGlobal = 1, kLocal = 2 };

// One queued alignment as the DP kernels see it.  "rows" is the sequence
// streamed down the DP rows, "cols" the one held in the per-lane profile.
struct PairDesc {
  int64_t row_off;  // offset of the row sequence in its buffer
  int64_t col_off;  // offset of the column sequence in its buffer
  int32_t m;        // number of rows (>= 1)
  int32_t n;        // number of columns (>= 1)
  int32_t pair;     // index of the score in scores_out
  int32_t flags;    // kTransposed: rows come from B, columns from A
};
constexpr int32_t kTransposed = 1;

// Full-DP variants (chosen per length bin, by default or by the autotuner):
// the packed 16-bit kernel, the 32-bit stripe kernel with K = 8, 16 or 32
// columns per lane, and the multi-wave wavefront.  Bits 8..15 of
// PairDesc::flags carry the variant of a 32-bit list item.
// kVarP16 (local mode): the 32-bit list's multi-stripe kernel with packed
// 16-bit cells, two pairs per group, int8 profiles of any alphabet in LDS,
// K = 8 columns per lane.
enum Variant : int32_t {
  kVarI16 = 0,
  kVarI32K8 = 1,
  kVarI32K16 = 2,
  kVarI32K32 = 3,
  kVarLong = 4,
  kVarP16 = 5,
  kNumVariants = 6
};
__host__ __device__ inline int variant_of(int32_t flags) { return (flags >> 8) & 0xFF; }
__host__ __device__ inline int32_t with_variant(int32_t flags, int v) { return (flags & ~0xFF00) | (v << 8); }
__host__ __device__ inline int variant_k(int v) {
  return (v == kVarI32K8 || v == kVarP16) ? 8 : (v == kVarI32K32 ? 32 : 16);
}
// Waves claim the 32-bit list in units of 8 items: two quads (one item per
// group each) or one octet of kVarP16 items (two per group); its length
// bins are padded to whole units.
constexpr int kClaim32 = 8;
// FP16 cells hold integers exactly up to 2048 in magnitude; the packed
// kernel keeps every value below this when it runs them
constexpr int kHalfLimit = 2048 - 64;
// Cell types of the packed full-DP kernel: int16 pairs, or FP16 pairs whose
// profile bytes are FP8 E4M3 codes (exact for the integers 0..16, one packed
// conversion per cell pair) or FP8 E5M2 codes (the upper byte of an FP16
// value, so v_perm alone builds the pair; exact for 0..8, 10, 12, 14, 16).
constexpr int kCellI16 = 0, kCellF16E4M3 = 1, kCellF16E5M2 = 2;

// FP8 E4M3 code (bias 7, 3 mantissa bits) of an integer 0..16
__host__ __device__ inline uint32_t fp8_e4m3(int v) {
  if (v <= 0) return 0u;
  int e = 0;
  while ((2 << e) <= v) ++e;
  const int mant = ((v << 3) >> e) & 7;
  return (uint32_t)(((e + 7) << 3) | mant);
}
// FP8 E5M2 code (bias 15, 2 mantissa bits: the upper byte of the FP16
// value) of an integer 0..16 that it holds exactly
__host__ __device__ inline uint32_t fp8_e5m2(int v) {
  if (v <= 0) return 0u;
  int e = 0;
  while ((2 << e) <= v) ++e;
  const int mant = ((v << 2) >> e) & 3;
  return (uint32_t)(((e + 15) << 2) | mant);
}
__host__ __device__ inline bool e5m2_exact(int v) { return v >= 0 && v <= 16 && (v <= 8 || v % 2 == 0); }

// Length bins: bin b holds pairs whose longer sequence has at most 64 << b
// residues (the last bin everything longer).
constexpr int kLenBins = 12;
__host__ __device__ inline int length_bin(int64_t longer) {
  int b = 0;
  while (b < kLenBins - 1 && longer > ((int64_t)64 << b)) ++b;
  return b;
}

// Status word bits, OR-ed by kernels; read back once per call.
constexpr int32_t kStatusBadOffsets = 1;
constexpr int32_t kStatusBadResidue = 2;
constexpr int32_t kStatusRange = 4;
constexpr int32_t kStatusStall = 8;   // a wavefront wait exceeded its spin limit
constexpr int32_t kStatusPlan = 32;   // a planned replay met a batch its buffers cannot hold

// Banded classes: 32-bit (band_class_width) and packed 16-bit
// (band16_class_width); banded rounds.
constexpr int kBandClasses = 10;
constexpr int kBand16Classes = 18;
constexpr int kMaxBandRounds = 8;

// Full-DP work lists: packed 16-bit, 32-bit stripes, 32-bit wavefront,
// packed 16-bit wavefront (global mode, two pairs per wave).
constexpr int kListSlots = 4;

// Cost classes of the 32-bit full-DP list inside a length bin: 8 classes of
// stripe count by 16 of row count, most stripes and rows first.  A wave's
// four pairs run their stripes in lockstep, each as long as the longest
// pair's, so the list is ordered by both, not by their product.
constexpr int kStripeClasses = 8;
constexpr int kRowClasses = 16;
constexpr int kCostClasses = kStripeClasses * kRowClasses;

// Work-list counters written by the classify kernel.
struct Counters {
  int32_t n_full32;      // items queued for the 32-bit full DP
  int32_t next_full32;   // work pointer of the persistent 32-bit kernel
  int32_t max_rows_multi;// largest m among multi-stripe items
  int32_t status;        // OR of kStatus* bits
  unsigned long long cells;  // sum of m*n over the batch
  int32_t n_full16;      // pairs queued for the packed 16-bit full DP
  int32_t next_full16;   // work pointer of the 16-bit kernel (in pairs)
  int32_t n_rerun32;     // 16-bit pairs that saturated, queued for 32 bits
  int32_t next_rerun32;  // work pointer of the re-run
  int32_t n_long;        // pairs queued for the multi-wave wavefront
  int32_t n_long_tasks;  // their stripes (one task per stripe)
  int32_t next_long;     // ticket counter of the wavefront kernel
  int32_t n_fallback;    // banded pairs sent to the full DP
  int32_t n_long16;      // pairs queued for the packed wavefront (consecutive pairs form duos)
  int32_t n_long16_tasks;  // their stripes (one task per duo stripe)
  int32_t next_long16;   // ticket counter of the packed wavefront kernel
  int32_t n_full32_pairs; // pairs in the 32-bit list (n_full32 less each bin's padding)
  long long long16_bnd_total;  // uint2 entries of all packed wavefront boundary columns
  long long long_bnd_total;  // int2 entries of all wavefront boundary columns
  // banded path: lists per round parity and lane-width class
  int32_t n_band[2][kBandClasses];
  int32_t next_band[kBandClasses];
  int32_t n_band16[2][kBand16Classes];   // packed 16-bit banded lists per round parity and class
  int32_t next_band16[kBand16Classes];
  int32_t band_accepted[8];  // pairs accepted in round r
  unsigned long long band_cells;  // cells computed by the banded kernels (both widths)
  unsigned long long band16_cells;  // of these, cells computed by the packed 16-bit kernel
  unsigned long long fallback_cells;  // sum of m*n over the fallback pairs
  unsigned long long route_cells[4];  // sum of m*n per full-DP list (16-bit, 32-bit, wavefront, packed wavefront)
  // length-binned lists: counts, offsets and scatter cursors per (list, bin)
  int32_t bin_count[kListSlots][kLenBins];
  int32_t bin_base[kListSlots][kLenBins];
  int32_t bin_cursor[kListSlots][kLenBins];
  int32_t bin_var32[kLenBins];   // 32-bit variant of each bin
  int32_t kmask32;               // K variants present in the 32-bit list
  unsigned long long bin_cells[kLenBins];  // sum of m*n of the routed pairs per bin
  // The 32-bit list inside each length bin, by cost class (largest first):
  // counts, offsets and scatter cursors.  Device-only: the host reads back
  // the counters up to kCountersHead.
  int32_t cost_count[2][kLenBins][kCostClasses];   // [0]: 32-bit list, [1]: packed wavefront list
  int32_t cost_base[2][kLenBins][kCostClasses];
  int32_t cost_cursor[2][kLenBins][kCostClasses];
};
constexpr size_t kCountersHead = offsetof(Counters, cost_count);

// ---- banded path ----
// Band widths (diagonals) of the banded kernel's classes: 16-lane groups
// with K = 4, 8, 12, 16, 24 columns per lane, then whole waves with K = 8,
// 12, 16, 20, 24.  Consecutive widths differ by at most 1.5x from 128 on.
__host__ __device__ inline int band_class_width(int kc) {
  return kc == 0 ? 64 : kc == 1 ? 128 : kc == 2 ? 192 : kc == 3 ? 256
       : kc == 4 ? 384 : kc == 5 ? 512 : kc == 6 ? 768 : kc == 7 ? 1024 : kc == 8 ? 1280 : 1536;
}
// Widest band of the raw entry point (every class), and of the exact entry
// point and the label search.
constexpr int kRawBandMax = 1536;
constexpr int kExactBandMax = 1024;

// Smallest class whose width holds B diagonals, or -1.
__host__ __device__ inline int band_class_for(int B) {
  for (int kc = 0; kc < kBandClasses; ++kc)
    if (band_class_width(kc) >= B) return kc;
  return -1;
}

// Upper bound on the score of every path that visits a diagonal outside
// [lo, hi] (lo <= min(0, n-m), hi >= max(0, n-m), 0 <= beta <= alpha).
// Returns false when no path can leave the band.
//  global: a path reaching diagonal hi+1 takes >= hi+1 horizontal and
//    >= hi+1-(n-m) vertical gap columns (it must return to n-m); one reaching
//    lo-1 takes >= 1-lo vertical and >= n-m-lo+1 horizontal ones.  With g
//    diagonal steps it has m+n-2g gap columns in >= 2 runs, so it scores at
//    most sigma_max*g - 2 alpha - beta*(m+n-2g-2), g <= (m+n-G)/2.
//  semi-global: a path through a cell of diagonal d has at most len(d)
//    diagonal steps and gaps cost >= 0: at most max(sigma_max,0)*len(d), and
//    len is largest on the nearest outside diagonals hi+1 and lo-1.
__host__ __device__ inline bool band_leave_bound(int m, int n, int lo, int hi, int sigma_max,
                                                 int alpha, int beta, int mode, int64_t *ub) {
  bool any = false;
  int64_t best = 0;
  if (mode == kGlobal) {
    int64_t G[2];
    int ng = 0;
    if (hi + 1 <= n) G[ng++] = 2LL * (hi + 1) - (n - m);
    if (lo - 1 >= -m) G[ng++] = (int64_t)(n - m) - 2LL * (lo - 1);
    for (int s = 0; s < ng; ++s) {
      const int64_t gmax = ((int64_t)m + n - G[s]) / 2;
      if ((int64_t)m + n - G[s] < 0) continue;
      const int64_t g = (sigma_max + 2 * beta >= 0) ? gmax : 0;
      const int64_t v = (int64_t)sigma_max * g - 2LL * alpha - (int64_t)beta * ((int64_t)m + n - 2 * g - 2);
      best = any ? (v > best ? v : best) : v;
      any = true;
    }
  } else {
    int64_t len = -1;
    if (hi + 1 <= n) {
      const int d = hi + 1;
      const int64_t l = d >= 0 ? (m < n - d ? m : n - d) : (m + d < n ? m + d : n);
      len = l > len ? l : len;
    }
    if (lo - 1 >= -m) {
      const int d = lo - 1;
      const int64_t l = d >= 0 ? (m < n - d ? m : n - d) : (m + d < n ? m + d : n);
      len = l > len ? l : len;
    }
    if (len >= 0) {
      any = true;
      best = (int64_t)(sigma_max > 0 ? sigma_max : 0) * len;
    }
  }
  *ub = best;
  return any;
}

// One banded pair: the orientation-fixed descriptor and its half-width.
struct BandItem {
  PairDesc d;
  int32_t w;
  int32_t pad_;
};

// Packed 16-bit banded classes (global mode): 64 << pc diagonals.
// Before each round every band list is sorted by row count, longest first,
// into one buffer (list l at sorted_base[l]): the pairs of one wave, and the
// two halves of a packed group, then run about the same number of wavefront
// steps.  Keys are 32-row buckets, the last one open.
constexpr int kBandLists = kBandClasses + kBand16Classes;  // 32-bit classes, then packed
constexpr int kSortBuckets = 512;
__host__ __device__ inline int sort_bucket(int m) { return (m >> 5) < kSortBuckets - 1 ? (m >> 5) : kSortBuckets - 1; }

struct BandArgs {
  const BandItem *sorted;   // this round's lists, sorted (the kernels read these)
  int64_t sorted_base[kBandLists];
  const uint8_t *seqs_a;
  const uint8_t *seqs_b;
  BandItem *lists;          // [2 parities][kBandClasses][list_cap] (requeued pairs go here)
  BandItem *lists16;        // [2 parities][kBand16Classes][list_cap] (packed 16-bit kernel)
  int64_t list_cap;
  int32_t pack16;           // 1: range-proven global pairs may use the packed kernel
  int32_t smax_pos;         // max(sigma_max, 0)
  int32_t drop16;           // max(0, -(sigma_min + 2 beta)) (packed range proof)
  Counters *ctr;
  const uint32_t *qwords;   // [2][32]: byte c of word r = sigma(r, c) + alpha + beta (row/col order)
  int32_t asz, alpha, beta, sigma_max;
  int32_t round, max_rounds;
  int32_t raw;              // 1: write the banded score, no rounds or fallback
  int32_t exact;            // 1: score exactly the diagonals of the requested half-width
  int32_t *scores;
  int32_t *lo_out, *hi_out; // optional: diagonal limits scored (A/B orientation)
  int32_t *accept_out;      // optional (raw): 1 if the certificate accepts the score
  PairDesc *fallback;       // rejected pairs for the full DP
};

hipError_t launch_band_dp_i32(int mode, int kc, const BandArgs &args, int grid, hipStream_t stream);
int band_dp_i32_blocks_per_cu(int mode, int kc);
int band_dp_i32_pairs_per_wave(int kc);
hipError_t launch_band_dp_i16(int pc, const BandArgs &args, int grid, hipStream_t stream);
int band_dp_i16_blocks_per_cu(int pc);
int band_dp_i16_pairs_per_wave(int pc);

// Packed classes (lane-group size x registers per lane): 16 x {5, 6, 7, 8,
// 10, 12, 14, 16}, then 64 x {5, 6, 7, 8, 10, 12, 14, 16, 20, 24}: widths
// 80..256 and 320..1536 diagonals, adjacent ones 1.14-1.25x apart.  No
// 64-diagonal class: with four registers per lane the step's fixed costs
// and dependency chain leave it at 0.35-0.41 of the packed peak against
// 0.60 for 80 diagonals, so the wider band is the faster one.
constexpr int kBand16Narrow = 8;  // classes on 16-lane groups
__host__ __device__ constexpr int band16_class_k(int pc) {
  const int k = pc < kBand16Narrow ? pc : pc - kBand16Narrow;  // the same K ladder on both
  return k == 0 ? 5 : k == 1 ? 6 : k == 2 ? 7 : k == 3 ? 8 : k == 4 ? 10 : k == 5 ? 12
       : k == 6 ? 14 : k == 7 ? 16 : k == 8 ? 20 : 24;
}
__host__ __device__ constexpr int band16_class_lanes(int pc) { return pc < kBand16Narrow ? kGroup : kWave; }
__host__ __device__ constexpr int band16_class_width(int pc) { return band16_class_lanes(pc) * band16_class_k(pc); }
__host__ __device__ inline int band16_class_for(int B) {
  for (int pc = 0; pc < kBand16Classes; ++pc)
    if (band16_class_width(pc) >= B) return pc;
  return -1;
}
// Every shifted cell of a W-diagonal band of an m x n global pair stays
// below sigma_max*min(m,n) + beta*(m + n + W) (columns run up to n + W),
// plus the score byte and margins; and above -(drop*min(m,n) + 3(alpha -
// beta)), drop = max(0, -(sigma_min + 2 beta)): the band holds the path
// that runs down diagonal 0 and then takes one gap run to the cell, and in
// the shifted frame a diagonal step adds sigma + 2 beta and a gap run costs
// alpha - beta.  The packed kernel stores a cell as its value plus a bias
// in an unsigned 16-bit number with 0 as -infinity (band16_bias), so the
// whole range, from the lower bound to the upper one, has to fit 65535.
__host__ __device__ inline int64_t band16_ub(int m, int n, int W, int smax_pos, int alpha, int beta) {
  const int64_t mn = m < n ? m : n;
  return (int64_t)smax_pos * mn + (int64_t)beta * ((int64_t)m + n + W) + alpha + 2 * beta + 256;
}
__host__ __device__ inline int64_t band16_lb(int m, int n, int drop, int alpha, int beta) {
  const int64_t mn = m < n ? m : n;
  return (int64_t)drop * mn + 3LL * (alpha - beta) + 256;
}
__host__ __device__ inline bool band16_range_ok(int m, int n, int W, int smax_pos, int drop, int alpha,
                                                int beta) {
  const int64_t ub = band16_ub(m, n, W, smax_pos, alpha, beta), lb = band16_lb(m, n, drop, alpha, beta);
  return lb < 32000 && ub + lb < 65000;
}
// Bias of a range-proven pair: 32768 when its upper bound leaves room, else
// as low as the upper bound needs (at least lb + 1 by the range proof), so
// every cell is stored in [1, 65280].
__host__ __device__ inline int band16_bias(int m, int n, int W, int smax_pos, int alpha, int beta) {
  const int64_t room = 65280 - band16_ub(m, n, W, smax_pos, alpha, beta);
  return room < 32768 ? (int)room : 32768;
}
// Whether a band of W diagonals is worth computing for an n-column pair
// instead of the full DP: a packed band at most 3/4 of the row (it costs
// about 0.6 W / n of the 32-bit full DP per attempt), a 32-bit band less
// than half of it.  Either way lo > -m and hi < n, so the band stays inside
// the matrix's diagonals.
__host__ __device__ inline bool band16_worth(int W, int n) { return 4 * W <= 3 * n; }
__host__ __device__ inline bool band32_worth(int W, int n) { return 2 * W < n; }
// Where a band request of half-width w for an m-row (shorter), n-column pair
// goes: a packed class (*packed = true), a 32-bit class, or -1 for the full
// DP (no class holds it, or it is not worth it).
__host__ __device__ inline int band_route(int m, int n, int w, bool pack16, int smax_pos, int drop, int alpha,
                                          int beta, bool *packed) {
  const int B = n - m + 2 * w + 1;
  if (pack16) {
    const int pc = band16_class_for(B);
    if (pc >= 0 && band16_worth(band16_class_width(pc), n) &&
        band16_range_ok(m, n, band16_class_width(pc), smax_pos, drop, alpha, beta)) {
      *packed = true;
      return pc;
    }
  }
  *packed = false;
  const int kc = band_class_for(B);
  if (kc < 0 || !band32_worth(band_class_width(kc), n)) return -1;
  return kc;
}
// Widest band (diagonals) a class may hold for an m-row, n-column pair
// (m <= n); 0 if none.
__host__ __device__ inline int band_widest(int m, int n, bool pack16, int smax_pos, int drop, int alpha,
                                           int beta) {
  int best = 0;
  for (int kc = 0; kc < kBandClasses; ++kc)
    if (band32_worth(band_class_width(kc), n) && band_class_width(kc) > best) best = band_class_width(kc);
  if (pack16)
    for (int pc = 0; pc < kBand16Classes; ++pc) {
      const int W = band16_class_width(pc);
      if (band16_worth(W, n) && W > best && band16_range_ok(m, n, W, smax_pos, drop, alpha, beta)) best = W;
    }
  return best;
}
// Half-width of the widest band for the pair, or -1 when no band is worth it.
__host__ __device__ inline int band_widest_w(int m, int n, bool pack16, int smax_pos, int drop, int alpha,
                                             int beta, int *W_out) {
  const int W = band_widest(m, n, pack16, smax_pos, drop, alpha, beta);
  *W_out = W;
  const int w = (W - (n - m) - 1) / 2;
  return (W > 0 && W >= n - m + 1) ? w : -1;
}
// Global mode: the smallest half-width w whose band of diagonals
// [min(0, n-m) - w, max(0, n-m) + w] has a leave bound (band_leave_bound) of
// at most `score`: sigma_max (min(m, n) - w - 1) - 2 alpha - beta (|n - m| +
// 2 w) <= score.  A band that contains the rejected one scores at least
// `score`, so it is accepted from this half-width on; when the rejected band
// held an optimal path this is exactly the pair's smallest accepted band.
// -1 when the bound does not shrink with w.
__host__ __device__ inline int band_w_for_score(int m, int n, int score, int sigma_max, int alpha, int beta) {
  const int64_t den = (int64_t)sigma_max + 2LL * beta;
  if (den <= 0) return -1;
  const int64_t mn = m < n ? m : n, dn = m < n ? n - m : m - n;
  const int64_t num = (int64_t)sigma_max * (mn - 1) - 2LL * alpha - (int64_t)beta * dn - score;
  if (num <= 0) return 0;
  const int64_t w = (num + den - 1) / den;
  return w < (1 << 30) ? (int)w : (1 << 30);
}

// A rejected band (this round computed W_cur diagonals, banded score
// `score`): queue the pair for the next round.  Global mode takes the
// half-width at which the score would pass the certificate
// (band_w_for_score), semi-global doubles it.  When that band fits no class
// but a class wider than W_cur exists, the pair gets the widest band
// instead, unless (global) the score already shows that the widest band
// cannot pass with the same score; the full DP takes it when no wider band
// is left or the rounds are spent.
__device__ inline void band_requeue(const BandArgs &a, const PairDesc &d, int w, int mode, int W_cur, int score) {
  int w2 = w > 0 ? 2 * w : 1;
  const int wr = mode == kGlobal ? band_w_for_score(d.m, d.n, score, a.sigma_max, a.alpha, a.beta) : -1;
  if (wr > w) w2 = wr;
  bool packed = false;
  const bool p16 = a.pack16 && mode == kGlobal;
  int c = band_route(d.m, d.n, w2, p16, a.smax_pos, a.drop16, a.alpha, a.beta, &packed);
  if (c >= 0 && wr > w && (packed ? band16_class_width(c) : band_class_width(c)) <= W_cur) {
    // the computed band would not grow (class rounding): double instead
    w2 = 2 * w2;
    c = band_route(d.m, d.n, w2, p16, a.smax_pos, a.drop16, a.alpha, a.beta, &packed);
  }
  if (c < 0) {
    int Wmax = 0;
    const int wcap = band_widest_w(d.m, d.n, p16, a.smax_pos, a.drop16, a.alpha, a.beta, &Wmax);
    if (Wmax > W_cur && wcap > w && !(wr > wcap)) {
      w2 = wcap;
      c = band_route(d.m, d.n, w2, p16, a.smax_pos, a.drop16, a.alpha, a.beta, &packed);
    }
  }
  if (a.round + 1 >= a.max_rounds || c < 0) {
    a.fallback[atomicAdd(&a.ctr->n_fallback, 1)] = d;
    return;
  }
  BandItem nb;
  nb.d = d;
  nb.w = w2;
  nb.pad_ = 0;
  const int nxt = (a.round & 1) ^ 1;
  if (packed) {
    const int slot = atomicAdd(&a.ctr->n_band16[nxt][c], 1);
    a.lists16[((int64_t)(nxt * kBand16Classes + c)) * a.list_cap + slot] = nb;
  } else {
    const int slot = atomicAdd(&a.ctr->n_band[nxt][c], 1);
    a.lists[((int64_t)(nxt * kBandClasses + c)) * a.list_cap + slot] = nb;
  }
}

// ---- learned band ----
constexpr int kMlpInputs = 32;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpInputs * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden + 1;  // 6337
constexpr int kMlpPartialStride = 6400;     // floats per gradient partial
constexpr int kMlpMaxParts = 256;           // gradient partials (one per wave) per step

hipError_t launch_features(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                           const int64_t *offs_b, int64_t n_pairs, float *out, int32_t *status,
                           int num_cu, hipStream_t stream);
hipError_t launch_mlp_predict(const float *params, const float *features, int64_t n, int32_t *w_out,
                              float *y_out, int num_cu, hipStream_t stream);
int mlp_grad_parts(int batch);

// Banded driver shared by the banded entry points (runtime.hip): raw = 1
// scores one band per pair (no rounds, no fallback), exact = 1 scores the
// requested diagonals themselves and skips pairs with a negative half-width.
int band_call(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b, const int64_t *offs_b,
              int64_t n_pairs, const as_scoring *scoring, int32_t mode, const int32_t *band_w,
              int32_t max_rounds, int32_t raw, int32_t exact, int32_t *scores_out, int32_t *lo_out,
              int32_t *hi_out, int32_t *accept_out, as_band_stats *stats, void *stream_ptr);
bool timing_enabled();
void release_learned_workspace();
void release_traceback_workspace();
void record_learned_timing(float features_ms, float mlp_ms);
void get_last_timing(as_timing *t);   // the timing record of the last call (no lock)
void set_last_timing(const as_timing &t);
hipError_t launch_mlp_train_step(const float *features, const int32_t *labels, const int32_t *order,
                                 int32_t batch, float tau, float *params, float *m1, float *m2,
                                 float *partials, float *grads_out, float lr, float c1, float c2,
                                 hipStream_t stream);

// A long pair and where its stripes and boundary columns live.
struct LongItem {
  PairDesc d;
  int32_t task0;     // ticket of its first stripe
  int32_t stripes;   // number of stripes (tasks)
  int64_t bnd_off;   // first boundary entry (int2) of its (stripes-1) columns
};

struct LongDpArgs {
  const uint8_t *seqs_a;
  const uint8_t *seqs_b;
  const LongItem *items;
  Counters *ctr;
  const int8_t *subst;
  int32_t asz;
  int32_t alpha;
  int32_t beta;
  int32_t *scores;
  int2 *bnd;       // boundary columns, (m+1) rows per stripe edge
  int32_t *flags;  // rows published per stripe, zeroed before launch
};

hipError_t launch_long_dp_i32(int mode, const LongDpArgs &args, int grid, hipStream_t stream);

// Packed 16-bit wavefront (global mode): duos of consecutive list items.
struct Long16Args {
  const uint8_t *seqs_a;
  const uint8_t *seqs_b;
  const LongItem *items;    // duo d: items 2d, 2d+1; item 2d holds the duo's task0, stripes, bnd_off
  Counters *ctr;
  const int8_t *subst;      // sigma, asz x asz row-major (at most 4 letters)
  int32_t asz, alpha, beta;
  int32_t *scores;
  uint2 *bnd;               // boundary columns, (max(m0, m1) + 1) rows per stripe edge
  int32_t *flags;           // rows published per task, zeroed before launch
};
hipError_t launch_long_dp_i16(const Long16Args &args, int grid, hipStream_t stream);
int long_dp_i16_blocks_per_cu();
int long_dp_i16_stripe_width();
constexpr int kLong16Width = 1024;  // columns per packed wavefront stripe (64 lanes x 16)
// Rows from which the automatic routing takes the packed wavefront: its
// 63-step pipeline fill per stripe is then at most 6% of the stripe, and it
// runs faster than the 32-bit stripe kernel from there on.
constexpr int kLong16MinRows = 1024;
// A global pair whose every shifted cell provably fits int16 (columns past n
// only lower cells, so the full matrix bound holds for the padded stripes).
__host__ __device__ inline bool long16_range_ok(int64_t m, int64_t n, int smax_pos, int alpha, int beta) {
  const int64_t ub = (int64_t)smax_pos * (m < n ? m : n) + (int64_t)beta * (m + n) + alpha + 2 * beta + 256;
  const int64_t lb = 3LL * (alpha - beta) + 256;
  return ub < 32000 && lb < 32000;
}
int long_dp_i32_blocks_per_cu(int mode, int asz);
int long_dp_i32_stripe_width(int asz);  // 64 K columns, K = 16 (alphabets <= 4) or 8
size_t long_dp_i32_lds_bytes(int asz);

struct FullDpArgs {
  const uint8_t *seqs_a;
  const uint8_t *seqs_b;
  const PairDesc *items;
  const int32_t *n_items;  // device: number of items in the list
  int32_t *next;           // device: work pointer (starts at 0)
  Counters *ctr;
  const int8_t *subst;  // device copy, sigma(a, b) = subst[a * asz + b]
  int32_t asz;
  int32_t alpha;
  int32_t beta;
  int32_t *scores;
  int2 *bnd;            // boundary columns, one slot per group: 2 * bnd_rows int2
  int64_t bnd_rows;     // rows per boundary buffer (>= max_rows_multi + 1)
  PairDesc *rerun;      // kVarP16: pairs whose 16-bit maximum saturates (32-bit re-run)
  int32_t *n_rerun;
  int32_t sat_limit;
};

// Arguments of the packed 16-bit kernel: two pairs per 16-lane group, one in
// each half of every 32-bit register.
struct FullDp16Args {
  const uint8_t *seqs_a;
  const uint8_t *seqs_b;
  const PairDesc *items;   // 16-bit work list (pairs; consecutive pairs share a group)
  Counters *ctr;
  PairDesc *rerun;         // saturated pairs are appended here for the 32-bit kernel
  const int8_t *subst;
  int32_t asz;             // <= 4 (profile held in registers, one byte per residue)
  int32_t alpha;
  int32_t beta;
  int32_t sat_limit;       // local: a 16-bit maximum >= this is re-run with 32 bits
  int32_t *scores;
  int32_t half;            // cell type: kCellI16, or FP16 cells (values within +-2048)
};

hipError_t launch_full_dp_i16(int mode, const FullDp16Args &args, int grid, hipStream_t stream);

// All-against-all batches on the packed kernel (columns of at most one
// packed stripe, alphabet of at most 4): row sequence q against column
// sequence c, score at scores[q * ld + c] (tr = 0) or scores[c * ld + q]
// (tr = 1: the caller's first set is the column set, and sigma's first
// index is the column letter).
struct AllVsAllArgs {
  const uint8_t *seqs_r;   // row sequences
  const int64_t *offs_r;   // [n_rows + 1]
  const uint8_t *seqs_c;   // column sequences
  const int64_t *offs_c;   // [n_cols + 1]
  int32_t n_rows, n_cols;
  int32_t rows_per_block;  // row sequences per work item (a multiple of 8)
  int32_t n_blocks;        // ceil(n_rows / rows_per_block)
  int32_t tr;
  int64_t ld;              // leading dimension of scores
  const int8_t *subst;
  int32_t asz, alpha, beta, sat_limit;
  int32_t *scores;
  int32_t *next;           // work counter (items = column x block)
  int32_t *status;
  PairDesc *rerun;         // saturated local pairs for the 32-bit kernel
  int32_t *n_rerun;
  int32_t half;            // cell type (kCellI16, or FP16 cells: values within +-2048)
  int32_t kcols;           // columns per lane: 8, 16 or 32 (stripes of 128, 256 or 512 columns)
  int32_t eq_rows;         // > 0: every row sequence has this length (global calls stream them)
};
// Longest column sequence the all-against-all packed kernel takes.
constexpr int kAvsaMaxCols = 512;
hipError_t launch_all_vs_all_i16(int mode, const AllVsAllArgs &args, int grid, hipStream_t stream);
int all_vs_all_i16_blocks_per_cu(int mode, int kcols);
int full_dp_i16_blocks_per_cu(int mode);
int full_dp_i16_stripe_width();

// Launch the persistent 32-bit full-DP kernel for `mode` on `grid` blocks
// of one wave each; kmask is the set of K variants the list holds (bit 0:
// K = 8, bit 1: 16, bit 2: 32).  Returns hipSuccess or the launch error.
hipError_t launch_full_dp_i32(int mode, const FullDpArgs &args, int kmask, int grid, hipStream_t stream);
// Resident one-wave blocks per CU for that instantiation (occupancy query).
int full_dp_i32_blocks_per_cu(int mode, int asz, int kmask);
// Columns per stripe (16 lanes x K).
int full_dp_i32_stripe_width(int k);
size_t full_dp_i32_lds_bytes(int asz, int kmask);
__host__ __device__ inline int kmask_of_variant(int v) {
  return v == kVarI32K8 ? 1 : (v == kVarI32K32 ? 4 : (v == kVarP16 ? 8 : 2));
}

}  // namespace asmi
