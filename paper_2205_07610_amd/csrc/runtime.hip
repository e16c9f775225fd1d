// Host runtime and C ABI of the library (include/anyseq_mi.h).
//
// Full DP (as_align_batch), on the caller's stream:
//   1. classify: per pair, offsets are validated, empty pairs are scored by
//      their closed form (mode paragraphs of the paper's section 2.1), every
//      other pair gets an orientation (which sequence runs down the rows) and
//      a route -- packed 16-bit list, 32-bit list or multi-wave wavefront --
//      after the a priori range checks;
//   2. the counters are read back (one small device-to-host copy);
//   3. the persistent kernels drain the lists; 16-bit pairs that saturate are
//      re-queued and recomputed with 32-bit cells;
//   4. the status word is read back and turned into the return code.
// Banded path (as_align_batch_band): the band classify step queues every pair
// with its initial half-width by lane-width class; each round the banded
// kernel either accepts a pair (certificate), re-queues it with the band
// doubled, or sends it to the full-DP fallback list, which then goes through
// the full-DP routing of step 1 and steps 3-4.
#include <algorithm>
#include <mutex>
#include <string.h>
#include <vector>

#include "internal.h"
#include "anyseq_mi.h"

namespace asmi {
namespace {

constexpr int64_t kMaxLen = (int64_t)1 << 30;
constexpr int64_t kCellBudget32 = (int64_t)1 << 28;  // |shifted cell| must stay below
constexpr int32_t kStatusArg = 16;                    // band wider than the widest class

struct RouteParams {
  int64_t n_pairs;
  int32_t mode, alpha, beta, smax_abs, smax_pos;
  int32_t drop16;         // max(0, -(sigma_min + 2 beta)): the banded int16 range proof
  int32_t allow16;        // the scoring fits the packed kernel's byte profile
  int32_t allowP16;       // local mode, sigma + alpha fits a byte: the packed LDS-profile variant
  int32_t half;           // the packed kernel runs FP16 cells (range bound below 2048)
  int32_t long_w;         // stripe width of the wavefront kernel
  int32_t long_min_rows;  // automatic routing: rows needed for the wavefront
  int32_t long16;         // global range-proven wavefront pairs may take the packed wavefront
  int32_t only_bin;       // -1, or the one length bin to route (autotuning)
  int8_t var_of_bin[kLenBins];        // variant per length bin, -1 = automatic
  int32_t sample_stride[kLenBins];    // route every stride-th pair of a bin (1: all)
};

// Work lists of the full DP, by kernel.
enum List { kList16 = 0, kList32 = 1, kListLong = 2, kListLong16 = 3, kLists = kListSlots };
// lists ordered by cost class inside each bin (index into the cost arrays), or -1
__host__ __device__ inline int cost_list(int l) { return l == kList32 ? 0 : (l == kListLong16 ? 1 : -1); }

// Orientation minimising the stripe passes of a 32-bit kernel with stripes
// of W columns: a pass costs (rows + 15) steps.
__device__ inline bool orient_rows_b(int64_t m, int64_t n, int W) {
  const int64_t sa = (n + W - 1) / W, sb = (m + W - 1) / W;
  return sb * (n + kGroup - 1) < sa * (m + kGroup - 1);
}

__device__ inline void fill_desc(PairDesc &d, bool tr, int64_t a0, int64_t m, int64_t b0, int64_t n,
                                 int64_t p, int var) {
  d.row_off = tr ? b0 : a0;
  d.col_off = tr ? a0 : b0;
  d.m = (int32_t)(tr ? n : m);
  d.n = (int32_t)(tr ? m : n);
  d.pair = (int32_t)p;
  d.flags = with_variant(tr ? kTransposed : 0, var);
}

// List, length bin and descriptor of a non-empty pair (A at a0, length m;
// B at b0, length n), or -1 when the pair is not routed (autotuning runs
// route one bin, or a sample of it).  A bin's variant applies to the pairs
// it can serve; the others take the automatic rule: packed 16-bit when the
// shorter side fits one packed stripe and the range is proven (or local:
// saturation is detected at run time), the wavefront for pairs with many
// rows (the packed one from 1024, the 32-bit one from 2048) and more than
// one wavefront stripe, else 32-bit stripes of 256.
__device__ int route_pair(const RouteParams &c, int64_t a0, int64_t m, int64_t b0, int64_t n, int64_t p,
                          PairDesc &d, int &bin) {
  bin = length_bin(m > n ? m : n);
  if (c.only_bin >= 0 && bin != c.only_bin) return -1;
  if (c.sample_stride[bin] > 1 && p % c.sample_stride[bin] != 0) return -1;
  const int v = c.var_of_bin[bin];
  if (v == kVarI32K8 || v == kVarI32K16 || v == kVarI32K32 || (v == kVarP16 && c.allowP16)) {
    fill_desc(d, orient_rows_b(m, n, kGroup * variant_k(v)), a0, m, b0, n, p, v);
    return kList32;
  }
  const bool tr = orient_rows_b(m, n, kGroup * 16);
  fill_desc(d, tr, a0, m, b0, n, p, kVarI32K16);
  if ((v < 0 || v == kVarI16) && c.allow16 && d.n <= kGroup * 16 && c.half) {
    // FP16 cells: local maxima are checked at run time against a threshold
    // below 2048; global and semi-global cells stay below
    // sigma_max*256 + beta*(rows + 512) + alpha + 2 beta + 16, a bound that
    // grows with the rows only, so it also covers the rows one pair of a
    // group runs past its own end while its partner continues
    if (c.mode == kLocal) return kList16;
    const int64_t ub = (int64_t)c.smax_pos * (kGroup * 16) + (int64_t)c.beta * (d.m + 2 * kGroup * 16) +
                       c.alpha + 2 * c.beta + 16;
    if (ub < kHalfLimit) return kList16;
  } else if ((v < 0 || v == kVarI16) && c.allow16 && d.n <= kGroup * 16) {
    if (c.mode == kLocal) return kList16;
    // shifted-frame cells stay below sigma_max*min(m,n) + beta*(m+n), plus
    // the profile byte and the padding offset beta*256
    const int64_t ub = (int64_t)c.smax_pos * (m < n ? m : n) + (int64_t)c.beta * (m + n) +
                       (int64_t)c.beta * (kGroup * 16) + c.alpha + 2 * c.beta + 256;
    if (ub < 32000) return kList16;
  }
  if (d.n > c.long_w && (v == kVarLong || v < 0)) {
    if (c.long16 && c.mode == kGlobal && c.allow16 && (v == kVarLong || d.m >= kLong16MinRows) &&
        long16_range_ok(m, n, c.smax_pos, c.alpha, c.beta))
      return kListLong16;
    if (v == kVarLong || d.m >= c.long_min_rows) return kListLong;
  }
  if (c.allowP16)  // local pairs of the 32-bit list: packed cells, LDS profiles
    fill_desc(d, orient_rows_b(m, n, kGroup * variant_k(kVarP16)), a0, m, b0, n, p, kVarP16);
  return kList32;
}

// Validation shared by the classify kernels.  Returns false for pairs that
// need no DP (errors, empty sequences -- scored here).
__device__ bool check_pair(const RouteParams &c, const int64_t *offs_a, const int64_t *offs_b,
                           int64_t p, Counters *ctr, int32_t *scores, bool first_pass, int64_t &a0,
                           int64_t &m, int64_t &b0, int64_t &n) {
  a0 = offs_a[p];
  b0 = offs_b[p];
  const int64_t a1 = offs_a[p + 1], b1 = offs_b[p + 1];
  m = a1 - a0;
  n = b1 - b0;
  if (a0 < 0 || b0 < 0 || a1 < a0 || b1 < b0) {
    if (first_pass) atomicOr(&ctr->status, kStatusBadOffsets);
    return false;
  }
  // Every cell value, in either frame the kernels use, is bounded in
  // magnitude by (|sigma|max + alpha + 2 beta) * (m + n + 2).
  if (m >= kMaxLen || n >= kMaxLen ||
      (int64_t)(c.smax_abs + c.alpha + 2 * c.beta) * (m + n + 2) >= kCellBudget32) {
    if (first_pass) atomicOr(&ctr->status, kStatusRange);
    return false;
  }
  if (m == 0 || n == 0) {
    // one gap of length m + n (global) or the empty alignment (others)
    const int64_t len = m + n;
    if (first_pass)
      scores[p] = (c.mode == kGlobal && len > 0) ? (int32_t)(-c.alpha - c.beta * (len - 1)) : 0;
    return false;
  }
  return true;
}

// A pair of the source: from the offsets (validated, empty pairs scored) or
// from a list of descriptors (the banded path's fallback, already valid).
__device__ bool source_pair(const RouteParams &c, const int64_t *offs_a, const int64_t *offs_b,
                            const PairDesc *src, int64_t i, Counters *ctr, int32_t *scores, bool first,
                            int64_t &a0, int64_t &m, int64_t &b0, int64_t &n, int64_t &p) {
  if (!src) {
    p = i;
    return check_pair(c, offs_a, offs_b, i, ctr, scores, first, a0, m, b0, n);
  }
  const PairDesc f = src[i];
  const bool tr = (f.flags & kTransposed) != 0;
  a0 = tr ? f.col_off : f.row_off;
  b0 = tr ? f.row_off : f.col_off;
  m = tr ? f.n : f.m;
  n = tr ? f.m : f.n;
  p = f.pair;
  return true;
}

// Block-level list reservation: pass 1 counts the routes of the block's
// pairs in LDS, one global atomic per route reserves the block's slices, pass
// 2 recomputes the routes and scatters through LDS cursors.
template <int R>
struct BlockLists {
  int cnt[R];
  int base[R];
  unsigned long long cells;
  unsigned long long rcells[R];  // m*n per route
};

__device__ inline unsigned long long valid_cells(int64_t a0, int64_t m, int64_t b0, int64_t n) {
  return (a0 >= 0 && b0 >= 0 && m > 0 && n > 0) ? (unsigned long long)(m * n) : 0ull;
}

__device__ inline int64_t source_count(const RouteParams &c, const PairDesc *src, const Counters *ctr) {
  return src ? (int64_t)ctr->n_fallback : c.n_pairs;
}

// Classification, step 1 of 3: per (list, length bin) counts, cells, the
// 32-bit variant of every bin and the longest multi-stripe row count.
// Cost class of an item of an ordered list inside its length bin (0 =
// costliest): stripe class (32-bit list: the stripe count, exact up to 8
// stripes, else 8 even ranges; packed wavefront list: 8 even ranges of the
// column count) by row class (16 even ranges of the bin's longest side).
__device__ inline int cost_class(const PairDesc &d, int bin, int l) {
  const int64_t longer = (int64_t)64 << bin;                // the bin's longest side
  int64_t st;
  if (l == kListLong16) {
    // column class: 8 even ranges of the bin's longest side, so the duos of
    // a class share their stripe count and use at most four stripe widths
    st = kStripeClasses - 1 - (int64_t)d.n * kStripeClasses / (longer + 1);
  } else {
    const int ws = kGroup * variant_k(variant_of(d.flags));  // stripe width
    const int64_t smax = (longer + ws - 1) / ws;
    st = smax - ((int64_t)d.n + ws - 1) / ws;               // 0 = most stripes
    if (smax > kStripeClasses) st = st * kStripeClasses / smax;
  }
  st = st < 0 ? 0 : (st >= kStripeClasses ? kStripeClasses - 1 : st);
  int64_t rc = kRowClasses - 1 - (int64_t)d.m * kRowClasses / (longer + 1);  // 0 = most rows
  rc = rc < 0 ? 0 : (rc >= kRowClasses ? kRowClasses - 1 : rc);
  return (int)(st * kRowClasses + rc);
}

__global__ void __launch_bounds__(256) route_count_kernel(RouteParams c, const int64_t *offs_a,
                                                          const int64_t *offs_b, const PairDesc *src,
                                                          Counters *ctr, int32_t *scores) {
  constexpr int R = kLists * kLenBins;
  constexpr int RC = kLenBins * kCostClasses;
  __shared__ int cnt[R];
  __shared__ int ccnt[2 * RC];
  __shared__ unsigned long long rcells[kLists];
  __shared__ unsigned long long bcells[kLenBins];
  __shared__ unsigned long long cells_sh;
  const int64_t total = source_count(c, src, ctr);
  const int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < total ? lo + chunk : total;
  for (int r = threadIdx.x; r < R; r += blockDim.x) cnt[r] = 0;
  for (int r = threadIdx.x; r < 2 * RC; r += blockDim.x) ccnt[r] = 0;
  if (threadIdx.x < kLists) rcells[threadIdx.x] = 0;
  if (threadIdx.x < kLenBins) bcells[threadIdx.x] = 0;
  if (threadIdx.x == 0) cells_sh = 0;
  __syncthreads();
  unsigned long long cells = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    int64_t a0, m, b0, n, p;
    const bool dp = source_pair(c, offs_a, offs_b, src, i, ctr, scores, true, a0, m, b0, n, p);
    cells += src ? (unsigned long long)(m * n) : valid_cells(a0, m, b0, n);
    if (!dp) continue;
    PairDesc d;
    int bin;
    const int l = route_pair(c, a0, m, b0, n, p, d, bin);
    if (l < 0) continue;
    atomicAdd(&cnt[l * kLenBins + bin], 1);
    atomicAdd(&rcells[l], (unsigned long long)(m * n));
    atomicAdd(&bcells[bin], (unsigned long long)(m * n));
    if (cost_list(l) >= 0) atomicAdd(&ccnt[cost_list(l) * RC + bin * kCostClasses + cost_class(d, bin, l)], 1);
    if (l == kList32) {
      ctr->bin_var32[bin] = variant_of(d.flags);  // the same for every pair of the bin
      // boundary rows: multi-stripe items, and every packed item (its group
      // partner may have more stripes, and the group exports the longer half's rows)
      if (d.n > kGroup * variant_k(variant_of(d.flags)) || variant_of(d.flags) == kVarP16)
        atomicMax(&ctr->max_rows_multi, d.m);
    }
  }
  atomicAdd(&cells_sh, cells);
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += blockDim.x)
    if (cnt[r]) atomicAdd(&ctr->bin_count[r / kLenBins][r % kLenBins], cnt[r]);
  for (int r = threadIdx.x; r < 2 * RC; r += blockDim.x)
    if (ccnt[r]) atomicAdd(&ctr->cost_count[r / RC][(r % RC) / kCostClasses][r % kCostClasses], ccnt[r]);
  if (threadIdx.x < kLists && rcells[threadIdx.x])
    atomicAdd(&ctr->route_cells[threadIdx.x], rcells[threadIdx.x]);
  if (threadIdx.x < kLenBins && bcells[threadIdx.x])
    atomicAdd(&ctr->bin_cells[threadIdx.x], bcells[threadIdx.x]);
  if (threadIdx.x == 0) {
    if (cells_sh) atomicAdd(src ? &ctr->fallback_cells : &ctr->cells, cells_sh);
  }
}

// Step 2 of 3 (one thread): list offsets of every bin, longest bins first;
// 32-bit bins are padded to whole claims of kClaim32 items (a wave never
// mixes variants) with items of pair -1.  Capacities (0 = unchecked) guard a planned replay: a
// batch that would overflow the plan's boundary buffer is refused.
__global__ void __launch_bounds__(kWave) route_scan_kernel(Counters *ctr, PairDesc *items32,
                                                            int64_t bnd_rows_cap) {
  static_assert(kCostClasses == 2 * kWave, "two cost classes per lane");
  if (blockIdx.x != 0) return;
  const int lane = threadIdx.x;
  int kmask = 0;
  int real32 = 0;
  for (int l = 0; l < kLists; ++l) {
    int base = 0;
    for (int b = kLenBins - 1; b >= 0; --b) {
      if (lane == 0) ctr->bin_base[l][b] = base;
      int cnt = ctr->bin_count[l][b];
      const int cl = cost_list(l);
      if (cl >= 0 && cnt > 0) {
        // cost classes of the bin, costliest first (a prefix sum over the
        // lanes, lane j holding classes 2j and 2j + 1)
        const int c0 = ctr->cost_count[cl][b][2 * lane], c1 = ctr->cost_count[cl][b][2 * lane + 1];
        int incl = c0 + c1;
#pragma unroll
        for (int dd = 1; dd < kWave; dd <<= 1) {
          const int y = __shfl_up(incl, dd);
          if (lane >= dd) incl += y;
        }
        const int first = base + incl - c0 - c1;
        ctr->cost_base[cl][b][2 * lane] = first;
        ctr->cost_base[cl][b][2 * lane + 1] = first + c0;
      }
      if (l == kList32 && cnt > 0) {
        real32 += cnt;
        const int padded = (cnt + kClaim32 - 1) / kClaim32 * kClaim32;
        const int v = ctr->bin_var32[b];
        if (lane < padded - cnt) {
          PairDesc d{0, 0, 0, 0, -1, with_variant(0, v)};
          items32[base + cnt + lane] = d;
        }
        kmask |= kmask_of_variant(v);
        cnt = padded;
      }
      base += cnt;
    }
    if (lane == 0) {
      if (l == kList16) ctr->n_full16 = base;
      else if (l == kList32) {
        ctr->n_full32 = base;
        ctr->n_full32_pairs = real32;
      }
      else if (l == kListLong) ctr->n_long = base;
      else ctr->n_long16 = base;
    }
  }
  if (lane != 0) return;
  ctr->kmask32 = kmask;
  if (bnd_rows_cap > 0 && ctr->n_full32 > 0 && (int64_t)ctr->max_rows_multi + 1 > bnd_rows_cap) {
    atomicOr(&ctr->status, kStatusPlan);
    ctr->n_full32 = ctr->n_full32_pairs = ctr->n_full16 = ctr->n_long = ctr->n_long16 = 0;
  }
}

// Step 3 of 3: scatter into the lists, each block reserving its slice of
// every (list, bin) with one atomic.
__global__ void __launch_bounds__(256) route_scatter_kernel(RouteParams c, const int64_t *offs_a,
                                                            const int64_t *offs_b, const PairDesc *src,
                                                            PairDesc *items16, PairDesc *items32,
                                                            LongItem *items_long, LongItem *items_long16,
                                                            Counters *ctr) {
  constexpr int R = kLists * kLenBins;
  constexpr int RC = kLenBins * kCostClasses;
  __shared__ int cnt[R];
  __shared__ int base[R];
  __shared__ int ccnt[2 * RC];
  __shared__ int cbase[2 * RC];
  if (ctr->status & kStatusPlan) return;
  const int64_t total = source_count(c, src, ctr);
  const int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < total ? lo + chunk : total;
  for (int r = threadIdx.x; r < R; r += blockDim.x) cnt[r] = 0;
  for (int r = threadIdx.x; r < 2 * RC; r += blockDim.x) ccnt[r] = 0;
  __syncthreads();
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    int64_t a0, m, b0, n, p;
    if (!source_pair(c, offs_a, offs_b, src, i, ctr, nullptr, false, a0, m, b0, n, p)) continue;
    PairDesc d;
    int bin;
    const int l = route_pair(c, a0, m, b0, n, p, d, bin);
    if (l < 0) continue;
    const int cl = cost_list(l);
    if (cl >= 0) atomicAdd(&ccnt[cl * RC + bin * kCostClasses + cost_class(d, bin, l)], 1);
    else atomicAdd(&cnt[l * kLenBins + bin], 1);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    const int l = r / kLenBins, b = r % kLenBins;
    base[r] = cnt[r] ? ctr->bin_base[l][b] + atomicAdd(&ctr->bin_cursor[l][b], cnt[r]) : 0;
    cnt[r] = 0;
  }
  for (int r = threadIdx.x; r < 2 * RC; r += blockDim.x) {
    const int cl = r / RC, b = (r % RC) / kCostClasses, k = r % kCostClasses;
    cbase[r] = ccnt[r] ? ctr->cost_base[cl][b][k] + atomicAdd(&ctr->cost_cursor[cl][b][k], ccnt[r]) : 0;
    ccnt[r] = 0;
  }
  __syncthreads();
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    int64_t a0, m, b0, n, p;
    if (!source_pair(c, offs_a, offs_b, src, i, ctr, nullptr, false, a0, m, b0, n, p)) continue;
    PairDesc d;
    int bin;
    const int l = route_pair(c, a0, m, b0, n, p, d, bin);
    if (l < 0) continue;
    const int cl = cost_list(l);
    if (cl >= 0) {
      const int r = cl * RC + bin * kCostClasses + cost_class(d, bin, l);
      const int slot = cbase[r] + atomicAdd(&ccnt[r], 1);
      if (l == kList32) items32[slot] = d;
      else items_long16[slot].d = d;
      continue;
    }
    const int r = l * kLenBins + bin;
    const int slot = base[r] + atomicAdd(&cnt[r], 1);
    if (l == kList16) items16[slot] = d;
    else items_long[slot].d = d;
  }
}

// Banded path entry: orientation (rows = the shorter sequence), initial
// half-width, lane-width class; pairs whose first band is already wider than
// the widest class, or than half the matrix, go straight to the fallback list.
// raw = 1 queues every pair in the class that holds its request (too wide a
// band is an error); with exact = 1 a negative half-width leaves the pair out.
__global__ void __launch_bounds__(256) band_classify_kernel(RouteParams c, const int64_t *offs_a,
                                                            const int64_t *offs_b, const int32_t *w0,
                                                            int32_t raw, int32_t exact, BandItem *lists,
                                                            BandItem *lists16, int32_t pack16,
                                                            int64_t list_cap, PairDesc *fallback,
                                                            Counters *ctr, int32_t *scores) {
  // routes: 32-bit classes, packed classes, then the fallback list
  constexpr int R = kBandClasses + kBand16Classes + 1;
  constexpr int kFall = kBandClasses + kBand16Classes;
  __shared__ BlockLists<R> bl;
  const int64_t chunk = (c.n_pairs + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < c.n_pairs ? lo + chunk : c.n_pairs;
  if (threadIdx.x < R) bl.cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) bl.cells = 0;
  __syncthreads();
  unsigned long long cells = 0;
  auto classify = [&](int64_t p, bool first, BandItem &bi) -> int {
    int64_t a0, m, b0, n;
    const bool dp = check_pair(c, offs_a, offs_b, p, ctr, scores, first, a0, m, b0, n);
    if (first) cells += valid_cells(a0, m, b0, n);
    if (!dp) return -1;
    const bool tr = n < m;
    bi.d.row_off = tr ? b0 : a0;
    bi.d.col_off = tr ? a0 : b0;
    bi.d.m = (int32_t)(tr ? n : m);
    bi.d.n = (int32_t)(tr ? m : n);
    bi.d.pair = (int32_t)p;
    bi.d.flags = tr ? kTransposed : 0;
    int w = w0[p];
    if (exact && w < 0) return -1;
    w = w < 0 ? 0 : (w > (1 << 20) ? (1 << 20) : w);
    bi.w = w;
    bi.pad_ = 0;
    if (raw) {
      const int B = bi.d.n - bi.d.m + 2 * w + 1;
      if (B > (exact ? kExactBandMax : kRawBandMax)) {
        if (first) atomicOr(&ctr->status, kStatusArg);
        return -1;
      }
      // raw scores come from the kernel the rounds would use: the packed one
      // when the range proof holds for the class that fits the request
      if (pack16) {
        const int pc = band16_class_for(B);
        if (pc >= 0 && band16_range_ok(bi.d.m, bi.d.n, band16_class_width(pc), c.smax_pos, c.drop16, c.alpha,
                                       c.beta))
          return kBandClasses + pc;
      }
      return band_class_for(B);
    }
    bool packed = false;
    int rc = band_route(bi.d.m, bi.d.n, w, pack16 != 0, c.smax_pos, c.drop16, c.alpha, c.beta, &packed);
    if (rc < 0) {  // no class holds the request: start from the widest band instead
      int Wmax = 0;
      const int wcap = band_widest_w(bi.d.m, bi.d.n, pack16 != 0, c.smax_pos, c.drop16, c.alpha, c.beta, &Wmax);
      if (wcap < 0) return kFall;
      bi.w = wcap;
      rc = band_route(bi.d.m, bi.d.n, wcap, pack16 != 0, c.smax_pos, c.drop16, c.alpha, c.beta, &packed);
      if (rc < 0) return kFall;
    }
    return packed ? kBandClasses + rc : rc;
  };
  for (int64_t p = lo + threadIdx.x; p < hi; p += blockDim.x) {
    BandItem bi;
    const int r = classify(p, true, bi);
    if (r >= 0) atomicAdd(&bl.cnt[r], 1);
  }
  atomicAdd(&bl.cells, cells);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int kc = 0; kc < kBandClasses; ++kc)
      bl.base[kc] = bl.cnt[kc] ? atomicAdd(&ctr->n_band[0][kc], bl.cnt[kc]) : 0;
    for (int pc = 0; pc < kBand16Classes; ++pc)
      bl.base[kBandClasses + pc] =
          bl.cnt[kBandClasses + pc] ? atomicAdd(&ctr->n_band16[0][pc], bl.cnt[kBandClasses + pc]) : 0;
    bl.base[kFall] = bl.cnt[kFall] ? atomicAdd(&ctr->n_fallback, bl.cnt[kFall]) : 0;
    if (bl.cells) atomicAdd(&ctr->cells, bl.cells);
    for (int r = 0; r < R; ++r) bl.cnt[r] = 0;
  }
  __syncthreads();
  for (int64_t p = lo + threadIdx.x; p < hi; p += blockDim.x) {
    BandItem bi;
    const int r = classify(p, false, bi);
    if (r < 0) continue;
    const int slot = bl.base[r] + atomicAdd(&bl.cnt[r], 1);
    if (r == kFall) fallback[slot] = bi.d;
    else if (r >= kBandClasses) lists16[(int64_t)(r - kBandClasses) * list_cap + slot] = bi;
    else lists[(int64_t)r * list_cap + slot] = bi;
  }
}

// One block: the packed wavefront's duos (items 2d, 2d+1): stripes
// max(S0, S1), first ticket and boundary offset of each duo (prefix sums).
__global__ void __launch_bounds__(256) long16_prep_kernel(LongItem *items, Counters *ctr) {
  __shared__ int sst[256];
  __shared__ long long sbe[256];
  const int n = ctr->n_long16;
  const int nd = (n + 1) / 2;
  int task = 0;
  long long bnd = 0;
  for (int b = 0; b < nd; b += 256) {
    const int i = b + threadIdx.x;
    int st = 0;
    long long be = 0;
    if (i < nd) {
      const PairDesc d0 = items[2 * i].d;
      int S = (d0.n + kLong16Width - 1) / kLong16Width, mm = d0.m;
      if (2 * i + 1 < n) {
        const PairDesc d1 = items[2 * i + 1].d;
        S = max(S, (d1.n + kLong16Width - 1) / kLong16Width);
        mm = max(mm, d1.m);
      }
      st = S;
      be = (long long)(S - 1) * (mm + 1);
    }
    sst[threadIdx.x] = st;
    sbe[threadIdx.x] = be;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int vs = threadIdx.x >= off ? sst[threadIdx.x - off] : 0;
      const long long vb = threadIdx.x >= off ? sbe[threadIdx.x - off] : 0;
      __syncthreads();
      sst[threadIdx.x] += vs;
      sbe[threadIdx.x] += vb;
      __syncthreads();
    }
    if (i < nd) {
      items[2 * i].task0 = task + sst[threadIdx.x] - st;
      items[2 * i].stripes = st;
      items[2 * i].bnd_off = bnd + sbe[threadIdx.x] - be;
    }
    task += sst[255];
    bnd += sbe[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctr->n_long16_tasks = task;
    ctr->long16_bnd_total = bnd;
  }
}

// ---- sorting the band lists by row count (before each round) ----
// The lists of one round, as one virtual sequence: list l holds n[l] items
// at src[l] and goes to out[base[l] .. base[l] + n[l]).
struct SortLists {
  const BandItem *src[kBandLists];
  int32_t n[kBandLists];
  int64_t base[kBandLists];
  int64_t total;
};

__device__ inline int sort_list_of(const SortLists &s, int64_t g) {
  int l = 0;
  while (l < kBandLists - 1 && g >= s.base[l] + s.n[l]) ++l;
  return l;
}

// Histogram of (list, bucket) over the round's items: per block in LDS, then
// one global atomic per non-zero bin.
__global__ void __launch_bounds__(256) band_sort_count_kernel(SortLists s, int32_t *hist) {
  __shared__ int32_t h[kBandLists * kSortBuckets];
  for (int i = threadIdx.x; i < kBandLists * kSortBuckets; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < s.total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int l = sort_list_of(s, g);
    const int m = s.src[l][g - s.base[l]].d.m;
    atomicAdd(&h[l * kSortBuckets + sort_bucket(m)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBandLists * kSortBuckets; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// One wave per list turns its histogram into the first slot of each bucket,
// largest bucket first (lane j owns 8 consecutive buckets of that order).
constexpr int kSortScanThreads = 1024;
__global__ void __launch_bounds__(kSortScanThreads) band_sort_scan_kernel(SortLists s, int32_t *hist) {
  const int lane = threadIdx.x % kWave;
  constexpr int kPer = kSortBuckets / kWave;
  for (int l = threadIdx.x / kWave; l < kBandLists; l += kSortScanThreads / kWave) {
    int32_t *h = hist + l * kSortBuckets;
    int v[kPer];
    int sum = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      v[q] = h[kSortBuckets - 1 - (lane * kPer + q)];
      sum += v[q];
    }
    int incl = sum;  // inclusive prefix of the lanes' sums
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int y = __shfl_up(incl, d);
      if (lane >= d) incl += y;
    }
    int run = (int)s.base[l] + incl - sum;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      h[kSortBuckets - 1 - (lane * kPer + q)] = run;
      run += v[q];
    }
  }
}

// Each block takes a contiguous slice of the round's items, reserves its
// part of every (list, bucket) with one global atomic, and places the items.
__global__ void __launch_bounds__(256) band_sort_scatter_kernel(SortLists s, int32_t *cursor,
                                                                BandItem *out) {
  __shared__ int32_t h[kBandLists * kSortBuckets];
  const int64_t chunk = (s.total + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < s.total ? lo + chunk : s.total;
  for (int i = threadIdx.x; i < kBandLists * kSortBuckets; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int64_t g = lo + threadIdx.x; g < hi; g += blockDim.x) {
    const int l = sort_list_of(s, g);
    atomicAdd(&h[l * kSortBuckets + sort_bucket(s.src[l][g - s.base[l]].d.m)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBandLists * kSortBuckets; i += blockDim.x)
    if (h[i]) h[i] = atomicAdd(&cursor[i], h[i]);
  __syncthreads();
  for (int64_t g = lo + threadIdx.x; g < hi; g += blockDim.x) {
    const int l = sort_list_of(s, g);
    const BandItem bi = s.src[l][g - s.base[l]];
    out[atomicAdd(&h[l * kSortBuckets + sort_bucket(bi.d.m)], 1)] = bi;
  }
}

// One block: prefix sums over the wavefront list (first ticket and boundary
// offset of every long pair), and the score seed that the stripes' atomic
// maxima start from (0 = the empty alignment / boundary cells).
__global__ void __launch_bounds__(256) long_prep_kernel(LongItem *items, Counters *ctr, int32_t long_w,
                                                        int32_t mode, int32_t *scores, int64_t bnd_cap,
                                                        int64_t tasks_cap) {
  __shared__ int sst[256];
  __shared__ long long sbe[256];
  const int n = ctr->n_long;
  int task = 0;
  long long bnd = 0;
  for (int b = 0; b < n; b += 256) {
    const int i = b + threadIdx.x;
    int st = 0;
    long long be = 0;
    if (i < n) {
      const PairDesc d = items[i].d;
      st = (d.n + long_w - 1) / long_w;
      be = (long long)(st - 1) * (d.m + 1);
      if (mode != kGlobal) scores[d.pair] = 0;
    }
    sst[threadIdx.x] = st;
    sbe[threadIdx.x] = be;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int vs = threadIdx.x >= off ? sst[threadIdx.x - off] : 0;
      const long long vb = threadIdx.x >= off ? sbe[threadIdx.x - off] : 0;
      __syncthreads();
      sst[threadIdx.x] += vs;
      sbe[threadIdx.x] += vb;
      __syncthreads();
    }
    if (i < n) {
      items[i].task0 = task + sst[threadIdx.x] - st;
      items[i].stripes = st;
      items[i].bnd_off = bnd + sbe[threadIdx.x] - be;
    }
    task += sst[255];
    bnd += sbe[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctr->n_long_tasks = task;
    ctr->long_bnd_total = bnd;
    // a planned replay whose wavefront buffers are too small does no long work
    if ((bnd_cap > 0 && bnd > bnd_cap) || (tasks_cap > 0 && task > tasks_cap)) {
      atomicOr(&ctr->status, kStatusPlan);
      ctr->n_long = 0;
      ctr->n_long_tasks = 0;
    }
  }
}

__global__ void __launch_bounds__(256) fill_kernel(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// All-against-all pairs [f0, f1) of the flat index f = q * n_s + s as full-DP
// descriptors (rows from the first set, columns from the second); a pair
// with an empty side is scored here by its closed form.
__global__ void __launch_bounds__(256) all_pairs_desc_kernel(const int64_t *offs_q, const int64_t *offs_s,
                                                              int64_t n_s, int64_t f0, int64_t f1, int32_t mode,
                                                              int32_t alpha, int32_t beta, PairDesc *out,
                                                              Counters *ctr, int32_t *scores) {
  for (int64_t f = f0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < f1;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = f / n_s, s = f % n_s;
    const int64_t a0 = offs_q[q], m = offs_q[q + 1] - a0;
    const int64_t b0 = offs_s[s], n = offs_s[s + 1] - b0;
    if (m == 0 || n == 0) {
      scores[f] = (mode == kGlobal && m + n > 0) ? (int32_t)(-alpha - beta * (m + n - 1)) : 0;
      continue;
    }
    PairDesc d;
    d.row_off = a0;
    d.col_off = b0;
    d.m = (int32_t)m;
    d.n = (int32_t)n;
    d.pair = (int32_t)f;
    d.flags = 0;
    out[atomicAdd(&ctr->n_fallback, 1)] = d;
  }
}

constexpr int kSideStreams = 3;

struct Workspace {
  int device = -1;
  int num_cu = 0;
  PairDesc *items = nullptr;    // 32-bit work list
  int64_t items_cap = 0;
  PairDesc *items16 = nullptr;  // 16-bit work list
  int64_t items16_cap = 0;
  PairDesc *rerun = nullptr;    // saturated 16-bit pairs
  int64_t rerun_cap = 0;
  LongItem *items_long = nullptr;  // wavefront list
  int64_t items_long_cap = 0;
  LongItem *items_long16 = nullptr;  // packed wavefront list (duos)
  int64_t items_long16_cap = 0;
  uint2 *bnd_long16 = nullptr;       // packed wavefront boundary columns
  int64_t bnd_long16_cap = 0;
  int32_t *flags16 = nullptr;        // packed wavefront progress counters
  int64_t flags16_cap = 0;
  int2 *bnd_long = nullptr;        // wavefront boundary columns
  int64_t bnd_long_cap = 0;
  int32_t *flags = nullptr;        // wavefront progress counters
  int64_t flags_cap = 0;
  BandItem *band_lists = nullptr;  // [2][kBandClasses][cap]
  int64_t band_cap = 0;
  BandItem *band16_lists = nullptr;  // [2][kBand16Classes][cap]
  int64_t band16_cap = 0;
  BandItem *band_sorted = nullptr;   // one round's lists, sorted by rows
  int64_t band_sorted_cap = 0;
  int32_t *sort_hist = nullptr;      // [kBandLists][kSortBuckets]
  PairDesc *fallback = nullptr;
  int64_t fallback_cap = 0;
  uint32_t *qwords = nullptr;      // [2][32]
  Counters *ctr = nullptr;
  Counters *host_ctr = nullptr;  // pinned
  int8_t *subst = nullptr;       // 32*32 bytes
  int2 *bnd = nullptr;
  int64_t bnd_cap = 0;           // int2 elements
  int32_t *tune_scores = nullptr;  // scores written by autotuning runs
  int64_t tune_scores_cap = 0;
  hipEvent_t ev[16] = {};
  // side streams of the banded rounds (default priority): one round's class
  // launches run on them concurrently, so a launch's tail overlaps the next
  hipStream_t side[kSideStreams] = {};
  hipEvent_t side_ev[kSideStreams + 1] = {};
  // No-allocation calls: every buffer is carved from the device's static
  // scratch array; buffers the call sizes late come from `pool`.
  bool noalloc = false;
  char *pool = nullptr;
  int64_t pool_left = 0;
};

bool g_timing = false;
bool g_band16 = true;  // packed 16-bit banded kernel for eligible global pairs
// Full-DP variant per (mode, length bin); -1 = automatic routing.
int8_t g_variants[3][kLenBins] = {{-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1},
                                  {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1},
                                  {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1}};
int32_t g_i16_limit = 32767;
int g_half_cells = 2;   // packed kernel's FP16 cells: 0 never, 1 when admissible, 2 automatic
// The automatic setting's cell type per mode as the autotuner measured it:
// -1 not measured (the static rule decides), 0 int16, 1 FP16.
int8_t g_half_pref[3] = {-1, -1, -1};
as_timing g_last_timing;

std::mutex g_lock;
std::vector<Workspace> g_ws;

#define AS_HIP(call)                         \
  do {                                       \
    if ((call) != hipSuccess) return AS_ERR_HIP; \
  } while (0)

int init_workspace(Workspace &w, int dev) {
  hipDeviceProp_t prop;
  AS_HIP(hipGetDeviceProperties(&prop, dev));
  w.num_cu = prop.multiProcessorCount;
  AS_HIP(hipMalloc(&w.ctr, sizeof(Counters)));
  AS_HIP(hipHostMalloc(&w.host_ctr, sizeof(Counters), hipHostMallocDefault));
  AS_HIP(hipMalloc(&w.subst, 32 * 32));
  AS_HIP(hipMalloc(&w.qwords, 2 * 32 * sizeof(uint32_t)));
  AS_HIP(hipMalloc(&w.sort_hist, kBandLists * kSortBuckets * sizeof(int32_t)));
  for (auto &e : w.ev) AS_HIP(hipEventCreate(&e));
  for (auto &st : w.side) AS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  for (auto &e : w.side_ev) AS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  w.device = dev;
  return AS_OK;
}

void free_workspace(Workspace &w) {
  void *bufs[] = {w.items, w.items16, w.rerun, w.items_long, w.bnd_long, w.flags, w.items_long16,
                  w.bnd_long16, w.flags16, w.band_lists,
                  w.band16_lists, w.band_sorted, w.sort_hist, w.fallback, w.qwords, w.ctr, w.subst, w.bnd,
                  w.tune_scores};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (w.host_ctr) (void)hipHostFree(w.host_ctr);
  for (auto &e : w.ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &st : w.side)
    if (st) (void)hipStreamDestroy(st);
  for (auto &e : w.side_ev)
    if (e) (void)hipEventDestroy(e);
  w = Workspace();
}

int get_workspace(Workspace **out) {
  int dev = 0;
  AS_HIP(hipGetDevice(&dev));
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  Workspace &w = g_ws[dev];
  if (w.device < 0) {
    int rc = init_workspace(w, dev);
    if (rc) return rc;
  }
  *out = &w;
  return AS_OK;
}

int grow(void **ptr, int64_t *cap, int64_t need, size_t elem) {
  if (*cap >= need) return AS_OK;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  const int64_t n = need + need / 4;
  AS_HIP(hipMalloc(ptr, (size_t)n * elem));
  *cap = n;
  return AS_OK;
}

// grow() for the buffers that run_full_lists sizes from the counters; a
// no-allocation workspace carves them from its pool instead (AS_ERR_SCRATCH
// when the pool cannot hold them).
int ws_grow(Workspace *w, void **ptr, int64_t *cap, int64_t need, size_t elem) {
  if (!w->noalloc) return grow(ptr, cap, need, elem);
  if (*cap >= need) return AS_OK;
  const int64_t bytes = ((need * (int64_t)elem) + 255) & ~(int64_t)255;
  if (bytes > w->pool_left) return AS_ERR_SCRATCH;
  *ptr = w->pool;
  *cap = need;
  w->pool += bytes;
  w->pool_left -= bytes;
  return AS_OK;
}

// Fill n int32 words with v on the stream (a kernel, not a memset node).
int fill_async(int32_t *p, int64_t n, int32_t v, hipStream_t stream) {
  if (n <= 0) return AS_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
  AS_HIP(hipGetLastError());
  return AS_OK;
}

int status_to_code(int32_t st) {
  if (st & kStatusStall) return AS_ERR_HIP;
  if (st & kStatusBadOffsets) return AS_ERR_OFFSETS;
  if (st & kStatusBadResidue) return AS_ERR_RESIDUE;
  if (st & kStatusRange) return AS_ERR_RANGE;
  if (st & (kStatusArg | kStatusPlan)) return AS_ERR_ARG;
  return AS_OK;
}

int read_counters(Workspace *w, hipStream_t stream, Counters *c) {
  AS_HIP(hipMemcpyAsync(w->host_ctr, w->ctr, kCountersHead, hipMemcpyDeviceToHost, stream));
  AS_HIP(hipStreamSynchronize(stream));
  *c = *w->host_ctr;
  return AS_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.f;
  return ms;
}

struct CallScoring {
  int asz, alpha, beta, mode, smin, smax, smax_abs, allow16;
  int half;       // the packed kernel runs FP16 cells for this call
  int half_adm;   // the FP16 cell type the scoring admits (kCellI16: none)
};

// Host-side checks of the scoring scheme; fills cs.
int check_scoring(const as_scoring *scoring, int32_t mode, CallScoring *cs) {
  const int asz = scoring->alphabet_size;
  const int alpha = scoring->gap_open, beta = scoring->gap_extend;
  if (asz < 2 || asz > 32 || beta < 0 || alpha < beta || alpha > 10000 || mode < 0 || mode > 2)
    return AS_ERR_SCORING;
  int smin = 127, smax = -128;
  for (int i = 0; i < asz * asz; ++i) {
    smin = scoring->subst[i] < smin ? scoring->subst[i] : smin;
    smax = scoring->subst[i] > smax ? scoring->subst[i] : smax;
  }
  // The 32-bit kernels store sigma + bias as int8 (bias = alpha + beta, or
  // alpha for local; padding columns store the bias itself).
  const int bias = (mode == kLocal) ? alpha : alpha + beta;
  if (smax + bias > 127 || smin + bias < -128 || bias > 127) return AS_ERR_SCORING;
  cs->asz = asz;
  cs->alpha = alpha;
  cs->beta = beta;
  cs->mode = mode;
  cs->smin = smin;
  cs->smax = smax;
  cs->smax_abs = (smax > -smin) ? smax : -smin;
  // The packed kernel keeps sigma + bias as unsigned bytes in registers, one
  // byte per letter of an alphabet of at most four.
  cs->allow16 = (asz <= 4 && smin + bias >= 0 && smax + bias <= 255) ? 1 : 0;
  // FP16 cells take their profile bytes (sigma + bias and the padding
  // value) as FP8 codes: E5M2 when every one is exact in it, else E4M3,
  // exact for all integers 0..16.  Automatic selection takes them for local
  // calls with E5M2 bytes whose maxima cannot reach the FP16 threshold
  // (sigma_max * 256 + alpha + 16 below it), where they need fewer VALU
  // instructions per cell than int16 and never add a re-run.
  const int pad = (mode == kLocal) ? alpha : (mode == kGlobal ? alpha - beta : alpha + beta);
  bool e5 = e5m2_exact(pad);
  for (int i = 0; i < asz * asz; ++i) e5 = e5 && e5m2_exact(scoring->subst[i] + bias);
  const bool h_ok = cs->allow16 && smax + bias <= 16 && pad <= 16;
  const int smax_pos = smax > 0 ? smax : 0;
  const int pref = g_half_pref[mode];
  const bool want = g_half_cells == 1 ||
                    (g_half_cells == 2 && (pref >= 0 ? pref == 1
                                                     : mode == kLocal && e5 && smax_pos * 256 + alpha + 16 < kHalfLimit));
  cs->half_adm = h_ok ? (e5 ? kCellF16E5M2 : kCellF16E4M3) : kCellI16;
  cs->half = want ? cs->half_adm : kCellI16;
  return AS_OK;
}

// Local re-run threshold of the packed kernel: the int16 limit, and for
// FP16 cells at most kHalfLimit (the scores of a step are at most 16, so a
// maximum first reaching the threshold is still exact).
int32_t packed_sat_limit(const CallScoring &cs) {
  return (cs.half && cs.mode == kLocal && g_i16_limit > kHalfLimit) ? kHalfLimit : g_i16_limit;
}

int classify_blocks(int64_t n) {
  int64_t blocks = (n + 1023) / 1024;
  if (blocks > 1024) blocks = 1024;
  return blocks < 1 ? 1 : (int)blocks;
}

RouteParams route_params(const CallScoring &cs, int64_t n_pairs) {
  RouteParams rp;
  rp.n_pairs = n_pairs;
  rp.mode = cs.mode;
  rp.alpha = cs.alpha;
  rp.beta = cs.beta;
  rp.smax_abs = cs.smax_abs;
  rp.smax_pos = cs.smax > 0 ? cs.smax : 0;
  rp.drop16 = cs.smin + 2 * cs.beta < 0 ? -(cs.smin + 2 * cs.beta) : 0;
  rp.allow16 = cs.allow16;
  rp.allowP16 = (cs.mode == kLocal && cs.smin + cs.alpha >= 0 && cs.smax + cs.alpha <= 255) ? 1 : 0;
  rp.half = cs.half;
  rp.long_w = long_dp_i32_stripe_width(cs.asz);
  rp.long_min_rows = 2048;
  rp.long16 = 1;
  rp.only_bin = -1;
  for (int b = 0; b < kLenBins; ++b) {
    rp.var_of_bin[b] = g_variants[cs.mode][b];
    rp.sample_stride[b] = 1;
  }
  return rp;
}

// Classification (count, scan, scatter) of the pairs given by the offsets
// (src == nullptr) or of a descriptor list holding n_src pairs.
int launch_classify(Workspace *w, const RouteParams &rp, const int64_t *offs_a, const int64_t *offs_b,
                    const PairDesc *src, int64_t n_src, int32_t *scores, hipStream_t stream,
                    int64_t bnd_rows_cap = 0) {
  const int blocks = classify_blocks(n_src);
  hipLaunchKernelGGL(route_count_kernel, dim3(blocks), dim3(256), 0, stream, rp, offs_a, offs_b, src, w->ctr,
                     scores);
  AS_HIP(hipGetLastError());
  hipLaunchKernelGGL(route_scan_kernel, dim3(1), dim3(64), 0, stream, w->ctr, w->items, bnd_rows_cap);
  AS_HIP(hipGetLastError());
  hipLaunchKernelGGL(route_scatter_kernel, dim3(blocks), dim3(256), 0, stream, rp, offs_a, offs_b, src,
                     w->items16, w->items, w->items_long, w->items_long16, w->ctr);
  AS_HIP(hipGetLastError());
  return AS_OK;
}

int lists_capacity(Workspace *w, int64_t n_pairs) {
  int rc;
  // the 32-bit list pads each length bin to whole quads
  if ((rc = grow((void **)&w->items, &w->items_cap, n_pairs + kClaim32 * kLenBins, sizeof(PairDesc))))
    return rc;
  if ((rc = grow((void **)&w->items16, &w->items16_cap, n_pairs, sizeof(PairDesc)))) return rc;
  if ((rc = grow((void **)&w->rerun, &w->rerun_cap, n_pairs, sizeof(PairDesc)))) return rc;
  if ((rc = grow((void **)&w->items_long, &w->items_long_cap, n_pairs, sizeof(LongItem)))) return rc;
  if ((rc = grow((void **)&w->items_long16, &w->items_long16_cap, n_pairs, sizeof(LongItem)))) return rc;
  return AS_OK;
}

// Steps 3-4 for whatever the lists hold (counters c read after they were
// filled): wavefront prefix, 16-bit, 32-bit and wavefront kernels, then the
// 32-bit re-run of saturated 16-bit pairs.
int run_full_lists(Workspace *w, const CallScoring &cs, const uint8_t *seqs_a,
                   const uint8_t *seqs_b, int32_t *scores_out, hipStream_t stream, bool timing,
                   Counters c) {
  const int mode = cs.mode, asz = cs.asz;
  int rc;
  if (c.n_long16 > 0) {
    hipLaunchKernelGGL(long16_prep_kernel, dim3(1), dim3(256), 0, stream, w->items_long16, w->ctr);
    AS_HIP(hipGetLastError());
  }
  if (c.n_long > 0) {
    hipLaunchKernelGGL(long_prep_kernel, dim3(1), dim3(256), 0, stream, w->items_long, w->ctr,
                       long_dp_i32_stripe_width(asz), mode, scores_out, (int64_t)0, (int64_t)0);
    AS_HIP(hipGetLastError());
  }
  if (c.n_long > 0 || c.n_long16 > 0)
    if ((rc = read_counters(w, stream, &c))) return rc;
  if (w->noalloc) {
    // a no-allocation call takes the wavefront buffers from its pool before
    // the first DP launch, so a batch that does not fit is refused whole
    if (c.n_long > 0 &&
        ((rc = ws_grow(w, (void **)&w->bnd_long, &w->bnd_long_cap, c.long_bnd_total > 0 ? c.long_bnd_total : 1,
                       sizeof(int2))) ||
         (rc = ws_grow(w, (void **)&w->flags, &w->flags_cap, c.n_long_tasks, sizeof(int32_t)))))
      return rc;
    if (c.n_long16 > 0 &&
        ((rc = ws_grow(w, (void **)&w->bnd_long16, &w->bnd_long16_cap,
                       c.long16_bnd_total > 0 ? c.long16_bnd_total : 1, sizeof(uint2))) ||
         (rc = ws_grow(w, (void **)&w->flags16, &w->flags16_cap, c.n_long16_tasks, sizeof(int32_t)))))
      return rc;
  }
  if (c.n_full16 > 0) {
    const int bpc = full_dp_i16_blocks_per_cu(mode);
    int64_t grid = (int64_t)bpc * w->num_cu;
    const int64_t need = ((int64_t)c.n_full16 + 2 * kGroupsPerWave - 1) / (2 * kGroupsPerWave);
    if (grid > need) grid = need;
    FullDp16Args a16;
    a16.seqs_a = seqs_a;
    a16.seqs_b = seqs_b;
    a16.items = w->items16;
    a16.ctr = w->ctr;
    a16.rerun = w->rerun;
    a16.subst = w->subst;
    a16.asz = asz;
    a16.alpha = cs.alpha;
    a16.beta = cs.beta;
    a16.sat_limit = packed_sat_limit(cs);
    a16.scores = scores_out;
    a16.half = cs.half;
    if (timing) AS_HIP(hipEventRecord(w->ev[2], stream));
    AS_HIP(launch_full_dp_i16(mode, a16, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[3], stream));
  }
  FullDpArgs args;
  args.seqs_a = seqs_a;
  args.seqs_b = seqs_b;
  args.ctr = w->ctr;
  args.subst = w->subst;
  args.asz = asz;
  args.alpha = cs.alpha;
  args.beta = cs.beta;
  args.scores = scores_out;
  args.rerun = w->rerun;
  args.n_rerun = &w->ctr->n_rerun32;
  args.sat_limit = g_i16_limit;
  if (c.n_full32 > 0) {
    const int bpc = full_dp_i32_blocks_per_cu(mode, asz, c.kmask32);
    int64_t grid = (int64_t)bpc * w->num_cu;
    const int64_t need_waves = ((int64_t)c.n_full32 + kGroupsPerWave - 1) / kGroupsPerWave;
    if (grid > need_waves) grid = need_waves;
    const int64_t bnd_rows = c.max_rows_multi > 0 ? (int64_t)c.max_rows_multi + 1 : 1;
    if (w->noalloc) {
      // a smaller persistent grid drains the same list; its boundary rows
      // must fit what is left of the scratch pool
      const int64_t per_wave = (int64_t)kGroupsPerWave * 2 * bnd_rows * (int64_t)sizeof(int2);
      const int64_t fit = w->pool_left / per_wave;
      if (grid > fit) grid = fit > 0 ? fit : 1;
    }
    if ((rc = ws_grow(w, (void **)&w->bnd, &w->bnd_cap, grid * kGroupsPerWave * 2 * bnd_rows, sizeof(int2))))
      return rc;
    args.items = w->items;
    args.n_items = &w->ctr->n_full32;
    args.next = &w->ctr->next_full32;
    args.bnd = w->bnd;
    args.bnd_rows = bnd_rows;
    if (timing) AS_HIP(hipEventRecord(w->ev[4], stream));
    AS_HIP(launch_full_dp_i32(mode, args, c.kmask32, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[5], stream));
  }
  if (c.n_long > 0) {
    if ((rc = ws_grow(w, (void **)&w->bnd_long, &w->bnd_long_cap, c.long_bnd_total > 0 ? c.long_bnd_total : 1,
                      sizeof(int2))))
      return rc;
    if ((rc = ws_grow(w, (void **)&w->flags, &w->flags_cap, c.n_long_tasks, sizeof(int32_t)))) return rc;
    if ((rc = fill_async(w->flags, c.n_long_tasks, 0, stream))) return rc;
    const int bpc = long_dp_i32_blocks_per_cu(mode, asz);
    int64_t grid = (int64_t)bpc * w->num_cu;
    if (grid > c.n_long_tasks) grid = c.n_long_tasks;
    LongDpArgs la;
    la.seqs_a = seqs_a;
    la.seqs_b = seqs_b;
    la.items = w->items_long;
    la.ctr = w->ctr;
    la.subst = w->subst;
    la.asz = asz;
    la.alpha = cs.alpha;
    la.beta = cs.beta;
    la.scores = scores_out;
    la.bnd = w->bnd_long;
    la.flags = w->flags;
    if (timing) AS_HIP(hipEventRecord(w->ev[8], stream));
    AS_HIP(launch_long_dp_i32(mode, la, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[9], stream));
  }
  if (c.n_long16 > 0) {
    if ((rc = ws_grow(w, (void **)&w->bnd_long16, &w->bnd_long16_cap,
                      c.long16_bnd_total > 0 ? c.long16_bnd_total : 1, sizeof(uint2))))
      return rc;
    if ((rc = ws_grow(w, (void **)&w->flags16, &w->flags16_cap, c.n_long16_tasks, sizeof(int32_t)))) return rc;
    if ((rc = fill_async(w->flags16, c.n_long16_tasks, 0, stream))) return rc;
    int64_t grid = (int64_t)long_dp_i16_blocks_per_cu() * w->num_cu;
    if (grid > c.n_long16_tasks) grid = c.n_long16_tasks;
    Long16Args l16;
    l16.seqs_a = seqs_a;
    l16.seqs_b = seqs_b;
    l16.items = w->items_long16;
    l16.ctr = w->ctr;
    l16.subst = w->subst;
    l16.asz = asz;
    l16.alpha = cs.alpha;
    l16.beta = cs.beta;
    l16.scores = scores_out;
    l16.bnd = w->bnd_long16;
    l16.flags = w->flags16;
    if (timing) AS_HIP(hipEventRecord(w->ev[14], stream));
    AS_HIP(launch_long_dp_i16(l16, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[15], stream));
  }
  Counters c2;
  if ((rc = read_counters(w, stream, &c2))) return rc;
  g_last_timing.pairs_long16 += c.n_long16;
  g_last_timing.cells_long16 += (int64_t)c2.route_cells[kListLong16];
  if (timing && c.n_long16 > 0) g_last_timing.long16_ms += elapsed(w->ev[14], w->ev[15]);
  g_last_timing.pairs_full32 += c.n_full32_pairs;
  if (c.n_full32 > 0) g_last_timing.full32_variants |= c.kmask32;
  g_last_timing.pairs_full16 += c.n_full16;
  if (c.n_full16 > 0) g_last_timing.full16_cell_type = cs.half;
  g_last_timing.pairs_long += c.n_long;
  g_last_timing.cells_full32 += (int64_t)c2.route_cells[kList32];
  g_last_timing.cells_full16 += (int64_t)c2.route_cells[kList16];
  g_last_timing.cells_long += (int64_t)c2.route_cells[kListLong];
  if (timing && c.n_full16 > 0) g_last_timing.full16_ms += elapsed(w->ev[2], w->ev[3]);
  if (timing && c.n_full32 > 0) g_last_timing.full32_ms += elapsed(w->ev[4], w->ev[5]);
  if (timing && c.n_long > 0) g_last_timing.long_ms += elapsed(w->ev[8], w->ev[9]);
  if ((rc = status_to_code(c2.status))) return rc;

  // 32-bit re-run of the 16-bit pairs whose maximum saturated
  g_last_timing.pairs_rerun32 += c2.n_rerun32;
  if (c2.n_rerun32 > 0) {
    const int bpc = full_dp_i32_blocks_per_cu(mode, asz, kmask_of_variant(kVarI32K16));
    int64_t grid = (int64_t)bpc * w->num_cu;
    const int64_t need_waves = ((int64_t)c2.n_rerun32 + kGroupsPerWave - 1) / kGroupsPerWave;
    if (grid > need_waves) grid = need_waves;
    // re-run pairs of the packed full DP fit one 32-bit stripe; those of the
    // packed LDS variant (local mode) may span several stripes, with at most
    // max_rows_multi rows
    const int64_t rr = (mode == kLocal && c.max_rows_multi > 0) ? (int64_t)c.max_rows_multi + 1 : 1;
    if (w->noalloc) {
      const int64_t per_wave = (int64_t)kGroupsPerWave * 2 * rr * (int64_t)sizeof(int2);
      const int64_t fit = std::max((w->bnd_cap * (int64_t)sizeof(int2)) / per_wave, w->pool_left / per_wave);
      if (grid > fit) grid = fit > 0 ? fit : 1;
    }
    if ((rc = ws_grow(w, (void **)&w->bnd, &w->bnd_cap, grid * kGroupsPerWave * 2 * rr, sizeof(int2)))) return rc;
    args.items = w->rerun;
    args.n_items = &w->ctr->n_rerun32;
    args.next = &w->ctr->next_rerun32;
    args.bnd = w->bnd;
    args.bnd_rows = rr;
    if (timing) AS_HIP(hipEventRecord(w->ev[6], stream));
    AS_HIP(launch_full_dp_i32(mode, args, kmask_of_variant(kVarI32K16), (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[7], stream));
    Counters c3;
    if ((rc = read_counters(w, stream, &c3))) return rc;
    if (timing) g_last_timing.rerun32_ms += elapsed(w->ev[6], w->ev[7]);
    if ((rc = status_to_code(c3.status))) return rc;
  }
  return AS_OK;
}


// Score words of the banded kernel: byte c of word r is sigma(r, c) + alpha +
// beta with rows from A (table 0) or from B (table 1).
int upload_qwords(Workspace *w, const as_scoring *scoring, const CallScoring &cs, hipStream_t stream,
                  uint32_t *host_words) {
  for (int t = 0; t < 2; ++t)
    for (int r = 0; r < 32; ++r) {
      uint32_t word = 0;
      if (r < cs.asz)
        for (int c = 0; c < cs.asz; ++c) {
          const int sv = t == 0 ? scoring->subst[r * cs.asz + c] : scoring->subst[c * cs.asz + r];
          word |= (uint32_t)((sv + cs.alpha + cs.beta) & 0xFF) << (8 * c);
        }
      host_words[t * 32 + r] = word;
    }
  AS_HIP(hipMemcpyAsync(w->qwords, host_words, 64 * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
  AS_HIP(hipStreamSynchronize(stream));  // host_words lives on the caller's stack
  return AS_OK;
}

// Checks of the banded path on top of check_scoring.
int check_band_scoring(const CallScoring &cs) {
  if (cs.mode == kLocal) return AS_ERR_ARG;
  // one byte per letter, four letters, unsigned
  if (cs.asz > 4 || cs.smin + cs.alpha + cs.beta < 0 || cs.smax + cs.alpha + cs.beta > 255 ||
      cs.alpha + cs.beta > 255)
    return AS_ERR_SCORING;
  return AS_OK;
}

}  // namespace
}  // namespace asmi

using namespace asmi;

namespace asmi {
namespace {

// Steps 1-4 of the full DP on a workspace whose lists hold n_pairs items.
int align_full(Workspace *w, const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
               const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, const CallScoring &cs,
               int32_t *scores_out, hipStream_t stream, bool timing) {
  int rc;
  AS_HIP(hipMemcpyAsync(w->subst, scoring->subst, (size_t)cs.asz * cs.asz, hipMemcpyHostToDevice, stream));
  if ((rc = fill_async((int32_t *)w->ctr, (int64_t)(sizeof(Counters) / sizeof(int32_t)), 0, stream))) return rc;
  memset(&g_last_timing, 0, sizeof(g_last_timing));
  if (timing) AS_HIP(hipEventRecord(w->ev[0], stream));
  const RouteParams rp = route_params(cs, n_pairs);
  if ((rc = launch_classify(w, rp, offs_a, offs_b, nullptr, n_pairs, scores_out, stream))) return rc;
  if (timing) AS_HIP(hipEventRecord(w->ev[1], stream));
  Counters c;
  if ((rc = read_counters(w, stream, &c))) return rc;
  g_last_timing.cells = (int64_t)c.cells;
  if (timing) g_last_timing.classify_ms = elapsed(w->ev[0], w->ev[1]);
  if ((rc = status_to_code(c.status))) return rc;
  return run_full_lists(w, cs, seqs_a, seqs_b, scores_out, stream, timing, c);
}

// ---- the no-allocation entry point's scratch ----
// One static array per device (the code object's copy on that device); its
// device address comes from hipGetSymbolAddress once per device, and only
// that address is ever handed to kernels or copies.
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[AS_NOALLOC_SCRATCH_BYTES];
void *g_scratch_ptr[kMaxDevices] = {};
Counters g_noalloc_host_ctr;  // counter read-back target (host, static)

int scratch_address(int dev, char **out) {
  if (dev < 0 || dev >= kMaxDevices) return AS_ERR_ARG;
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return AS_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char *)g_scratch_ptr[dev];
  return AS_OK;
}

// Carve a no-allocation workspace out of the device's scratch array: the
// counters, the sigma matrix and the five work lists of n_pairs items; the
// rest is the pool for the boundary buffers run_full_lists sizes later.
int noalloc_workspace(Workspace *w, int dev, int64_t n_pairs) {
  char *base = nullptr;
  int rc;
  if ((rc = scratch_address(dev, &base))) return rc;
  hipDeviceProp_t prop;
  AS_HIP(hipGetDeviceProperties(&prop, dev));
  w->device = dev;
  w->num_cu = prop.multiProcessorCount;
  w->noalloc = true;
  w->pool = base;
  w->pool_left = AS_NOALLOC_SCRATCH_BYTES;
  w->host_ctr = &g_noalloc_host_ctr;
  int64_t cap_ctr = 0, cap_subst = 0;
  if ((rc = ws_grow(w, (void **)&w->ctr, &cap_ctr, 1, sizeof(Counters)))) return rc;
  if ((rc = ws_grow(w, (void **)&w->subst, &cap_subst, 32 * 32, 1))) return rc;
  if ((rc = ws_grow(w, (void **)&w->items, &w->items_cap, n_pairs + kClaim32 * kLenBins, sizeof(PairDesc))))
    return rc;
  if ((rc = ws_grow(w, (void **)&w->items16, &w->items16_cap, n_pairs, sizeof(PairDesc)))) return rc;
  if ((rc = ws_grow(w, (void **)&w->rerun, &w->rerun_cap, n_pairs, sizeof(PairDesc)))) return rc;
  if ((rc = ws_grow(w, (void **)&w->items_long, &w->items_long_cap, n_pairs, sizeof(LongItem)))) return rc;
  if ((rc = ws_grow(w, (void **)&w->items_long16, &w->items_long16_cap, n_pairs, sizeof(LongItem)))) return rc;
  return AS_OK;
}

}  // namespace
}  // namespace asmi

extern "C" int as_align_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                              const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                              int32_t mode, int32_t *scores_out, void *stream_ptr) {
  if (!scoring || !offs_a || !offs_b || !seqs_a || !seqs_b || !scores_out || !scoring->subst)
    return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1) return AS_ERR_ARG;
  CallScoring cs;
  int rc = check_scoring(scoring, mode, &cs);
  if (rc) return rc;
  if (n_pairs == 0) return AS_OK;

  std::lock_guard<std::mutex> guard(g_lock);
  Workspace *w = nullptr;
  if ((rc = get_workspace(&w))) return rc;
  if ((rc = lists_capacity(w, n_pairs))) return rc;
  return align_full(w, seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, cs, scores_out,
                    (hipStream_t)stream_ptr, g_timing);
}

extern "C" int as_align_all_vs_all(const uint8_t *seqs_q, const int64_t *offs_q, int64_t n_q,
                                   const uint8_t *seqs_s, const int64_t *offs_s, int64_t n_s,
                                   const as_scoring *scoring, int32_t mode, int32_t *scores_out,
                                   void *stream_ptr) {
  if (!scoring || !offs_q || !offs_s || !seqs_q || !seqs_s || !scores_out || !scoring->subst) return AS_ERR_NULL;
  if (n_q < 0 || n_s < 0 || (n_q > 0 && n_s > 0 && n_q * n_s >= ((int64_t)1 << 31) - 1)) return AS_ERR_ARG;
  CallScoring cs;
  int rc = check_scoring(scoring, mode, &cs);
  if (rc) return rc;
  if (n_q == 0 || n_s == 0) return AS_OK;
  const int64_t n_pairs = n_q * n_s;
  hipStream_t stream = (hipStream_t)stream_ptr;
  // the two sets' offsets on the host: validation, longest sequences
  std::vector<int64_t> oq((size_t)n_q + 1), os((size_t)n_s + 1);
  AS_HIP(hipMemcpyAsync(oq.data(), offs_q, sizeof(int64_t) * (n_q + 1), hipMemcpyDeviceToHost, stream));
  AS_HIP(hipMemcpyAsync(os.data(), offs_s, sizeof(int64_t) * (n_s + 1), hipMemcpyDeviceToHost, stream));
  AS_HIP(hipStreamSynchronize(stream));
  int64_t mq = 0, ms = 0;
  for (int64_t i = 0; i < n_q; ++i) {
    if (oq[i] < 0 || oq[i + 1] < oq[i]) return AS_ERR_OFFSETS;
    mq = std::max(mq, oq[i + 1] - oq[i]);
  }
  for (int64_t i = 0; i < n_s; ++i) {
    if (os[i] < 0 || os[i + 1] < os[i]) return AS_ERR_OFFSETS;
    ms = std::max(ms, os[i + 1] - os[i]);
  }
  // the longest pair exists (longest query against longest subject)
  if (mq >= kMaxLen || ms >= kMaxLen || (int64_t)(cs.smax_abs + cs.alpha + 2 * cs.beta) * (mq + ms + 2) >= kCellBudget32)
    return AS_ERR_RANGE;

  std::lock_guard<std::mutex> guard(g_lock);
  Workspace *w = nullptr;
  if ((rc = get_workspace(&w))) return rc;
  memset(&g_last_timing, 0, sizeof(g_last_timing));
  AS_HIP(hipMemcpyAsync(w->subst, scoring->subst, (size_t)cs.asz * cs.asz, hipMemcpyHostToDevice, stream));
  // the packed kernel with the column profile reused across rows: the
  // columns from a set whose longest sequence fits a packed stripe of 128,
  // 256 or 512 columns (K = 8, 16, 32 per lane), the one with fewer steps
  // (columns x stripe width x the other set's rows + 15 per sequence)
  const auto stripe_w = [](int64_t L) -> double { return L <= 128 ? 128.0 : (L <= 256 ? 256.0 : 512.0); };
  const double rows_q = (double)(oq[n_q] - oq[0]) + 15.0 * n_q, rows_s = (double)(os[n_s] - os[0]) + 15.0 * n_s;
  const double cost_s = ms <= kAvsaMaxCols ? (double)n_s * stripe_w(ms) * rows_q : 1e300;
  const double cost_q = mq <= kAvsaMaxCols ? (double)n_q * stripe_w(mq) * rows_s : 1e300;
  const bool cols_s = ms <= kAvsaMaxCols && cost_s <= cost_q;
  const bool cols_q = !cols_s && mq <= kAvsaMaxCols;
  const int64_t col_max = cols_s ? ms : mq;
  const int kcols = col_max <= 128 ? 8 : (col_max <= 256 ? 16 : 32);
  const int Wc = kGroup * kcols;
  bool fast = cs.allow16 && (cols_s || cols_q);
  if (fast && mode != kLocal) {
    const int64_t ub = (int64_t)std::max(cs.smax, 0) * std::min(mq, ms) + (int64_t)cs.beta * (mq + ms) +
                       (int64_t)cs.beta * Wc + cs.alpha + 2 * cs.beta + 256;
    fast = ub < 32000;
  }
  if (fast) {
    AllVsAllArgs a;
    a.tr = cols_s ? 0 : 1;
    a.seqs_r = cols_s ? seqs_q : seqs_s;
    a.offs_r = cols_s ? offs_q : offs_s;
    a.seqs_c = cols_s ? seqs_s : seqs_q;
    a.offs_c = cols_s ? offs_s : offs_q;
    a.n_rows = (int32_t)(cols_s ? n_q : n_s);
    a.n_cols = (int32_t)(cols_s ? n_s : n_q);
    a.ld = n_s;
    a.kcols = kcols;
    int64_t grid = (int64_t)all_vs_all_i16_blocks_per_cu(mode, kcols) * w->num_cu;
    // about eight work items (column, block of rows) per resident wave
    int64_t n_blocks = (8 * grid + a.n_cols - 1) / a.n_cols;
    n_blocks = std::max<int64_t>(1, std::min<int64_t>(n_blocks, (a.n_rows + 7) / 8));
    int64_t rpb = (a.n_rows + n_blocks - 1) / n_blocks;
    rpb = (rpb + 7) / 8 * 8;
    a.rows_per_block = (int32_t)rpb;
    a.n_blocks = (int32_t)((a.n_rows + rpb - 1) / rpb);
    // global calls whose row sequences all have one length stream them
    // through the kernel's pipeline (128- and 256-column stripes; the
    // virtual row count of a group stays far inside int)
    {
      const std::vector<int64_t> &orow = cols_s ? oq : os;
      int64_t lmin = orow[1] - orow[0], lmax = lmin;
      for (int64_t i = 1; i < a.n_rows; ++i) {
        const int64_t L = orow[i + 1] - orow[i];
        lmin = std::min(lmin, L);
        lmax = std::max(lmax, L);
      }
      a.eq_rows = (mode == kGlobal && kcols <= 16 && lmin == lmax && lmin > 0 &&
                   (rpb / 8 + 1) * lmax < ((int64_t)1 << 30))
                      ? (int32_t)lmax : 0;
    }
    const int64_t items = (int64_t)a.n_cols * a.n_blocks;
    if (grid > items) grid = items;
    a.subst = w->subst;
    a.asz = cs.asz;
    a.alpha = cs.alpha;
    a.beta = cs.beta;
    // FP16 cells when the call admits them: local pairs check their maxima at
    // run time; global and semi-global ones need the row bound of the packed
    // kernel's routing for the longest row sequence.  Every pair of the call
    // shares that bound, so the automatic choice also takes FP16 cells for
    // global and semi-global calls with E5M2-exact scores (no pair is sent
    // elsewhere by it).
    const int64_t rows_max = cols_s ? mq : ms;
    a.half = cs.half;
    if (a.half == kCellI16 && g_half_cells == 2 && cs.half_adm == kCellF16E5M2 && mode != kLocal) a.half = kCellF16E5M2;
    if (a.half != kCellI16 && mode != kLocal &&
        (int64_t)std::max(cs.smax, 0) * Wc + (int64_t)cs.beta * (rows_max + 2 * Wc) + cs.alpha + 2 * cs.beta + 16 >=
            kHalfLimit)
      a.half = kCellI16;
    a.sat_limit = a.half ? packed_sat_limit(cs) : g_i16_limit;
    a.scores = scores_out;
    a.next = &w->ctr->next_full16;
    a.status = &w->ctr->status;
    if ((rc = grow((void **)&w->rerun, &w->rerun_cap, n_pairs, sizeof(PairDesc)))) return rc;
    a.rerun = w->rerun;
    a.n_rerun = &w->ctr->n_rerun32;
    if ((rc = fill_async((int32_t *)w->ctr, (int64_t)(sizeof(Counters) / sizeof(int32_t)), 0, stream))) return rc;
    const bool timing = g_timing;
    if (timing) AS_HIP(hipEventRecord(w->ev[2], stream));
    AS_HIP(launch_all_vs_all_i16(mode, a, (int)grid, stream));
    if (timing) AS_HIP(hipEventRecord(w->ev[3], stream));
    Counters c;
    if ((rc = read_counters(w, stream, &c))) return rc;
    g_last_timing.cells = 0;
    for (int64_t i = 0; i < n_q; ++i) g_last_timing.cells += (oq[i + 1] - oq[i]) * (os[n_s] - os[0]);
    g_last_timing.pairs_full16 = n_pairs - c.n_rerun32;
    g_last_timing.full16_cell_type = a.half;
    g_last_timing.cells_full16 = g_last_timing.cells;
    if (timing) g_last_timing.full16_ms = elapsed(w->ev[2], w->ev[3]);
    if ((rc = status_to_code(c.status))) return rc;
    g_last_timing.pairs_rerun32 = c.n_rerun32;
    if (c.n_rerun32 > 0) {
      FullDpArgs args;
      args.seqs_a = a.tr ? a.seqs_c : a.seqs_r;   // see the re-run descriptors
      args.seqs_b = a.tr ? a.seqs_r : a.seqs_c;
      args.ctr = w->ctr;
      args.subst = w->subst;
      args.asz = cs.asz;
      args.alpha = cs.alpha;
      args.beta = cs.beta;
      args.scores = scores_out;
      args.rerun = nullptr;   // the re-run list holds 32-bit items only
      args.n_rerun = nullptr;
      args.sat_limit = 0;
      // re-run items are single-stripe: 256 columns, or 512 for the widest packed stripes
      const int rv = kcols == 32 ? kVarI32K32 : kVarI32K16;
      const int bpc = full_dp_i32_blocks_per_cu(mode, cs.asz, kmask_of_variant(rv));
      int64_t g2 = (int64_t)bpc * w->num_cu;
      const int64_t need_waves = ((int64_t)c.n_rerun32 + kGroupsPerWave - 1) / kGroupsPerWave;
      if (g2 > need_waves) g2 = need_waves;
      if ((rc = grow((void **)&w->bnd, &w->bnd_cap, g2 * kGroupsPerWave * 2, sizeof(int2)))) return rc;
      args.items = w->rerun;
      args.n_items = &w->ctr->n_rerun32;
      args.next = &w->ctr->next_rerun32;
      args.bnd = w->bnd;
      args.bnd_rows = 1;
      AS_HIP(launch_full_dp_i32(mode, args, kmask_of_variant(rv), (int)g2, stream));
      Counters c3;
      if ((rc = read_counters(w, stream, &c3))) return rc;
      if ((rc = status_to_code(c3.status))) return rc;
    }
    return AS_OK;
  }
  // every other case: the pairs as descriptors, in chunks, through the
  // full-DP routing and kernels
  const int64_t chunk = std::min<int64_t>(n_pairs, (int64_t)1 << 24);
  if ((rc = lists_capacity(w, chunk))) return rc;
  if ((rc = grow((void **)&w->fallback, &w->fallback_cap, chunk, sizeof(PairDesc)))) return rc;
  const RouteParams rp = route_params(cs, chunk);
  for (int64_t f0 = 0; f0 < n_pairs; f0 += chunk) {
    const int64_t f1 = std::min(n_pairs, f0 + chunk);
    if ((rc = fill_async((int32_t *)w->ctr, (int64_t)(sizeof(Counters) / sizeof(int32_t)), 0, stream))) return rc;
    int64_t blocks = (f1 - f0 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(all_pairs_desc_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, offs_q, offs_s, n_s, f0,
                       f1, mode, cs.alpha, cs.beta, w->fallback, w->ctr, scores_out);
    AS_HIP(hipGetLastError());
    Counters c;
    if ((rc = read_counters(w, stream, &c))) return rc;
    if (c.n_fallback == 0) continue;
    if ((rc = launch_classify(w, rp, nullptr, nullptr, w->fallback, c.n_fallback, scores_out, stream))) return rc;
    if ((rc = read_counters(w, stream, &c))) return rc;
    if ((rc = status_to_code(c.status))) return rc;
    if ((rc = run_full_lists(w, cs, seqs_q, seqs_s, scores_out, stream, g_timing, c))) return rc;
  }
  return AS_OK;
}

extern "C" int as_align_batch_noalloc(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                                      const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                                      int32_t mode, int32_t *scores_out, void *stream_ptr) {
  if (!scoring || !offs_a || !offs_b || !seqs_a || !seqs_b || !scores_out || !scoring->subst)
    return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1) return AS_ERR_ARG;
  CallScoring cs;
  int rc = check_scoring(scoring, mode, &cs);
  if (rc) return rc;
  if (n_pairs == 0) return AS_OK;

  std::lock_guard<std::mutex> guard(g_lock);
  int dev = 0;
  AS_HIP(hipGetDevice(&dev));
  Workspace w;  // no events, no side streams: timing stays off
  if ((rc = noalloc_workspace(&w, dev, n_pairs))) return rc;
  return align_full(&w, seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, cs, scores_out,
                    (hipStream_t)stream_ptr, false);
}

// One round's class launches of one kernel family (packed or 32-bit), largest
// work (pairs x width) first, spread over the side streams and joined back
// into `stream`: every launch is persistent and fills the GPU, so running
// them concurrently lets the next one take over the slots that a finishing
// launch's last waves leave idle.
int launch_band_round(Workspace *w, const BandArgs &ba, int mode, const Counters &c, int cur, bool packed,
                      hipStream_t stream) {
  struct Launch {
    int cls;
    int64_t work, grid;
  };
  Launch ls[kBandLists];
  int nl = 0;
  const int ncls = packed ? kBand16Classes : kBandClasses;
  for (int k = 0; k < ncls; ++k) {
    const int cnt = packed ? c.n_band16[cur][k] : c.n_band[cur][k];
    if (!cnt) continue;
    const int width = packed ? band16_class_width(k) : band_class_width(k);
    int64_t grid = (int64_t)(packed ? band_dp_i16_blocks_per_cu(k) : band_dp_i32_blocks_per_cu(mode, k)) *
                   w->num_cu;
    const int ppw = packed ? band_dp_i16_pairs_per_wave(k) : band_dp_i32_pairs_per_wave(k);
    const int64_t need = ((int64_t)cnt + ppw - 1) / ppw;
    if (grid > need) grid = need;
    Launch l{k, (int64_t)cnt * width, grid};
    int i = nl++;
    while (i > 0 && ls[i - 1].work < l.work) {
      ls[i] = ls[i - 1];
      --i;
    }
    ls[i] = l;
  }
  if (!nl) return AS_OK;
  const int ns = nl < kSideStreams ? nl : kSideStreams;
  AS_HIP(hipEventRecord(w->side_ev[kSideStreams], stream));
  for (int i = 0; i < ns; ++i) AS_HIP(hipStreamWaitEvent(w->side[i], w->side_ev[kSideStreams], 0));
  for (int i = 0; i < nl; ++i) {
    hipStream_t st = w->side[i % ns];
    if (packed) AS_HIP(launch_band_dp_i16(ls[i].cls, ba, (int)ls[i].grid, st));
    else AS_HIP(launch_band_dp_i32(mode, ls[i].cls, ba, (int)ls[i].grid, st));
  }
  for (int i = 0; i < ns; ++i) {
    AS_HIP(hipEventRecord(w->side_ev[i], w->side[i]));
    AS_HIP(hipStreamWaitEvent(stream, w->side_ev[i], 0));
  }
  return AS_OK;
}

// Banded entry points share everything up to the rounds.
int asmi::band_call(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                    const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                    const int32_t *band_w, int32_t max_rounds, int32_t raw, int32_t exact,
                    int32_t *scores_out, int32_t *lo_out, int32_t *hi_out, int32_t *accept_out,
                    as_band_stats *stats, void *stream_ptr) {
  if (!scoring || !offs_a || !offs_b || !seqs_a || !seqs_b || !scores_out || !scoring->subst || !band_w)
    return AS_ERR_NULL;
  if ((lo_out == nullptr) != (hi_out == nullptr)) return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1) return AS_ERR_ARG;
  if (!raw && (max_rounds < 1 || max_rounds > kMaxBandRounds)) return AS_ERR_ARG;
  CallScoring cs;
  int rc = check_scoring(scoring, mode, &cs);
  if (rc) return rc;
  if ((rc = check_band_scoring(cs))) return rc;
  if (stats) memset(stats, 0, sizeof(*stats));
  if (n_pairs == 0) return AS_OK;

  std::lock_guard<std::mutex> guard(g_lock);
  Workspace *w = nullptr;
  if ((rc = get_workspace(&w))) return rc;
  hipStream_t stream = (hipStream_t)stream_ptr;
  if ((rc = lists_capacity(w, n_pairs))) return rc;
  if ((rc = grow((void **)&w->band_lists, &w->band_cap, 2 * kBandClasses * n_pairs, sizeof(BandItem))))
    return rc;
  const int64_t list_cap = w->band_cap / (2 * kBandClasses);
  // the packed kernel serves range-proven global pairs, except in the exact
  // mode (it has no per-diagonal mask)
  const int pack16 = (!exact && mode == kGlobal && g_band16) ? 1 : 0;
  if (pack16 && (rc = grow((void **)&w->band16_lists, &w->band16_cap, 2 * kBand16Classes * list_cap,
                           sizeof(BandItem))))
    return rc;
  if ((rc = grow((void **)&w->fallback, &w->fallback_cap, n_pairs, sizeof(PairDesc)))) return rc;
  if ((rc = grow((void **)&w->band_sorted, &w->band_sorted_cap, n_pairs, sizeof(BandItem)))) return rc;
  uint32_t host_words[64];
  AS_HIP(hipMemcpyAsync(w->subst, scoring->subst, (size_t)cs.asz * cs.asz, hipMemcpyHostToDevice, stream));
  if ((rc = upload_qwords(w, scoring, cs, stream, host_words))) return rc;
  AS_HIP(hipMemsetAsync(w->ctr, 0, sizeof(Counters), stream));
  const bool timing = g_timing;
  memset(&g_last_timing, 0, sizeof(g_last_timing));
  if (timing) AS_HIP(hipEventRecord(w->ev[0], stream));
  const RouteParams rp = route_params(cs, n_pairs);
  hipLaunchKernelGGL(band_classify_kernel, dim3(classify_blocks(n_pairs)), dim3(256), 0, stream, rp,
                     offs_a, offs_b, band_w, raw, exact, w->band_lists, pack16 ? w->band16_lists : nullptr,
                     pack16, list_cap, w->fallback, w->ctr, scores_out);
  AS_HIP(hipGetLastError());
  if (timing) AS_HIP(hipEventRecord(w->ev[1], stream));
  Counters c;
  if ((rc = read_counters(w, stream, &c))) return rc;
  g_last_timing.cells = (int64_t)c.cells;
  if (timing) g_last_timing.classify_ms = elapsed(w->ev[0], w->ev[1]);
  if ((rc = status_to_code(c.status))) return rc;

  BandArgs ba;
  ba.seqs_a = seqs_a;
  ba.seqs_b = seqs_b;
  ba.lists = w->band_lists;
  ba.lists16 = pack16 ? w->band16_lists : nullptr;
  ba.pack16 = pack16;
  ba.smax_pos = cs.smax > 0 ? cs.smax : 0;
  ba.drop16 = cs.smin + 2 * cs.beta < 0 ? -(cs.smin + 2 * cs.beta) : 0;
  ba.list_cap = list_cap;
  ba.ctr = w->ctr;
  ba.qwords = w->qwords;
  ba.asz = cs.asz;
  ba.alpha = cs.alpha;
  ba.beta = cs.beta;
  ba.sigma_max = cs.smax;
  ba.max_rounds = raw ? 1 : max_rounds;
  ba.raw = raw;
  ba.exact = exact;
  ba.scores = scores_out;
  ba.lo_out = lo_out;
  ba.hi_out = hi_out;
  ba.accept_out = accept_out;
  ba.fallback = w->fallback;
  ba.sorted = w->band_sorted;
  int rounds = 0;
  float band_ms = 0.f, band16_ms = 0.f, sort_ms = 0.f;
  for (int r = 0; r < ba.max_rounds; ++r) {
    const int cur = r & 1;
    // this round's lists, sorted by rows into one buffer
    SortLists sl;
    int64_t total = 0;
    for (int l = 0; l < kBandLists; ++l) {
      const bool p16 = l >= kBandClasses;
      const int k = p16 ? l - kBandClasses : l;
      sl.n[l] = p16 ? c.n_band16[cur][k] : c.n_band[cur][k];
      sl.src[l] = p16 ? (pack16 ? w->band16_lists + (int64_t)(cur * kBand16Classes + k) * list_cap : nullptr)
                      : w->band_lists + (int64_t)(cur * kBandClasses + k) * list_cap;
      sl.base[l] = total;
      ba.sorted_base[l] = total;
      total += sl.n[l];
    }
    sl.total = total;
    if (!total) break;
    // (every pair is in at most one list per round, so total <= n_pairs)
    if ((rc = grow((void **)&w->band_sorted, &w->band_sorted_cap, total, sizeof(BandItem)))) return rc;
    ba.sorted = w->band_sorted;
    ba.round = r;
    if (timing) AS_HIP(hipEventRecord(w->ev[13], stream));
    AS_HIP(hipMemsetAsync(w->sort_hist, 0, kBandLists * kSortBuckets * sizeof(int32_t), stream));
    const int sort_blocks = (int)((total + 4095) / 4096);
    hipLaunchKernelGGL(band_sort_count_kernel, dim3(sort_blocks), dim3(256), 0, stream, sl, w->sort_hist);
    hipLaunchKernelGGL(band_sort_scan_kernel, dim3(1), dim3(kSortScanThreads), 0, stream, sl, w->sort_hist);
    hipLaunchKernelGGL(band_sort_scatter_kernel, dim3(sort_blocks), dim3(256), 0, stream, sl, w->sort_hist,
                       w->band_sorted);
    AS_HIP(hipGetLastError());
    if (timing) AS_HIP(hipEventRecord(w->ev[10], stream));
    if ((rc = launch_band_round(w, ba, mode, c, cur, true, stream))) return rc;
    if (timing) AS_HIP(hipEventRecord(w->ev[12], stream));
    if ((rc = launch_band_round(w, ba, mode, c, cur, false, stream))) return rc;
    if (timing) AS_HIP(hipEventRecord(w->ev[11], stream));
    // this round's lists are consumed: clear their counters and work pointers
    AS_HIP(hipMemsetAsync(&w->ctr->n_band[cur][0], 0, sizeof(int32_t) * kBandClasses, stream));
    AS_HIP(hipMemsetAsync(&w->ctr->next_band[0], 0, sizeof(int32_t) * kBandClasses, stream));
    AS_HIP(hipMemsetAsync(&w->ctr->n_band16[cur][0], 0, sizeof(int32_t) * kBand16Classes, stream));
    AS_HIP(hipMemsetAsync(&w->ctr->next_band16[0], 0, sizeof(int32_t) * kBand16Classes, stream));
    if ((rc = read_counters(w, stream, &c))) return rc;
    if (timing) band_ms += elapsed(w->ev[10], w->ev[11]);
    if (timing) band16_ms += elapsed(w->ev[10], w->ev[12]);
    if (timing) sort_ms += elapsed(w->ev[13], w->ev[10]);
    if ((rc = status_to_code(c.status))) return rc;
    rounds = r + 1;
  }
  g_last_timing.band_ms = band_ms;
  g_last_timing.band16_ms = band16_ms;
  g_last_timing.classify_ms += sort_ms;
  g_last_timing.pairs_fallback = c.n_fallback;
  if (stats) {
    stats->rounds = rounds;
    for (int r = 0; r < kMaxBandRounds; ++r) stats->accepted[r] = c.band_accepted[r];
    stats->fallback = c.n_fallback;
    stats->band_cells = (int64_t)c.band_cells;
    stats->band16_cells = (int64_t)c.band16_cells;
    stats->cells = (int64_t)c.cells;
  }
  if (raw || c.n_fallback == 0) return AS_OK;

  // full DP for the fallback pairs
  if ((rc = launch_classify(w, rp, offs_a, offs_b, w->fallback, c.n_fallback, scores_out, stream))) return rc;
  if ((rc = read_counters(w, stream, &c))) return rc;
  if ((rc = status_to_code(c.status))) return rc;
  if (stats) stats->fallback_cells = (int64_t)c.fallback_cells;
  return run_full_lists(w, cs, seqs_a, seqs_b, scores_out, stream, timing, c);
}

extern "C" int as_align_batch_band(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                                   const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                                   int32_t mode, const int32_t *band_w0, int32_t max_rounds,
                                   int32_t *scores_out, as_band_stats *stats, void *stream) {
  return band_call(seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, mode, band_w0, max_rounds, 0, 0,
                   scores_out, nullptr, nullptr, nullptr, stats, stream);
}

extern "C" int as_band_scores(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                              const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                              int32_t mode, const int32_t *band_w, int32_t *scores_out,
                              int32_t *lo_out, int32_t *hi_out, void *stream) {
  return band_call(seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, mode, band_w, 1, 1, 0, scores_out,
                   lo_out, hi_out, nullptr, nullptr, stream);
}

extern "C" int as_band_certify(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                               const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                               int32_t mode, const int32_t *band_w, int32_t *scores_out,
                               int32_t *accept_out, void *stream) {
  if (!accept_out) return AS_ERR_NULL;
  return band_call(seqs_a, offs_a, seqs_b, offs_b, n_pairs, scoring, mode, band_w, 1, 1, 1, scores_out,
                   nullptr, nullptr, accept_out, nullptr, stream);
}

bool asmi::timing_enabled() { return g_timing; }

void asmi::record_learned_timing(float features_ms, float mlp_ms) {
  g_last_timing.features_ms = features_ms;
  g_last_timing.mlp_ms = mlp_ms;
}

void asmi::get_last_timing(as_timing *t) { *t = g_last_timing; }
void asmi::set_last_timing(const as_timing &t) { g_last_timing = t; }

// ---------------------------------------------------------------- plans
//
// A plan is one batch (its pointers, scoring and mode fixed) made
// replayable: it owns a private workspace sized by one planning run, and a
// HIP graph of the whole device-driven pipeline -- counters cleared by a
// fill kernel, classification, wavefront preparation and progress
// counters, the packed, 32-bit and wavefront kernels on fixed persistent
// grids (each reads its list length from device memory), the 32-bit re-run,
// and a copy of the counters to pinned host memory.  Nothing in it depends on
// the host between launches.  A replay whose inputs changed so much that the
// plan's boundary buffers cannot hold them is refused on the device
// (AS_ERR_ARG), never overrun.

struct PlanImpl {
  Workspace ws;
  CallScoring cs;
  RouteParams rp;
  const uint8_t *seqs_a, *seqs_b;
  const int64_t *offs_a, *offs_b;
  int64_t n_pairs;
  int32_t *scores;
  int kmask;
  int64_t bnd_rows, bnd_long_cap, flags_cap;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Enqueue the whole pipeline with fixed grids and no host synchronisation.
int enqueue_plan(PlanImpl &P, hipStream_t stream) {
  Workspace *w = &P.ws;
  const CallScoring &cs = P.cs;
  const int mode = cs.mode;
  const int n_words = (int)(sizeof(Counters) / sizeof(int32_t));
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, stream, (int32_t *)w->ctr, (int64_t)n_words, 0);
  AS_HIP(hipGetLastError());
  int rc = launch_classify(w, P.rp, P.offs_a, P.offs_b, nullptr, P.n_pairs, P.scores, stream, P.bnd_rows);
  if (rc) return rc;
  hipLaunchKernelGGL(long_prep_kernel, dim3(1), dim3(256), 0, stream, w->items_long, w->ctr,
                     long_dp_i32_stripe_width(cs.asz), mode, P.scores, P.bnd_long_cap, P.flags_cap);
  AS_HIP(hipGetLastError());
  hipLaunchKernelGGL(fill_kernel, dim3(64), dim3(256), 0, stream, w->flags, P.flags_cap, 0);
  AS_HIP(hipGetLastError());
  if (cs.allow16) {
    FullDp16Args a16;
    a16.seqs_a = P.seqs_a;
    a16.seqs_b = P.seqs_b;
    a16.items = w->items16;
    a16.ctr = w->ctr;
    a16.rerun = w->rerun;
    a16.subst = w->subst;
    a16.asz = cs.asz;
    a16.alpha = cs.alpha;
    a16.beta = cs.beta;
    a16.sat_limit = packed_sat_limit(cs);
    a16.scores = P.scores;
    a16.half = cs.half;
    AS_HIP(launch_full_dp_i16(mode, a16, full_dp_i16_blocks_per_cu(mode) * w->num_cu, stream));
  }
  FullDpArgs args;
  args.seqs_a = P.seqs_a;
  args.seqs_b = P.seqs_b;
  args.ctr = w->ctr;
  args.subst = w->subst;
  args.asz = cs.asz;
  args.alpha = cs.alpha;
  args.beta = cs.beta;
  args.scores = P.scores;
  args.rerun = w->rerun;
  args.n_rerun = &w->ctr->n_rerun32;
  args.sat_limit = g_i16_limit;
  args.items = w->items;
  args.n_items = &w->ctr->n_full32;
  args.next = &w->ctr->next_full32;
  args.bnd = w->bnd;
  args.bnd_rows = P.bnd_rows;
  const int grid32 = full_dp_i32_blocks_per_cu(mode, cs.asz, P.kmask) * w->num_cu;
  AS_HIP(launch_full_dp_i32(mode, args, P.kmask, grid32, stream));
  LongDpArgs la;
  la.seqs_a = P.seqs_a;
  la.seqs_b = P.seqs_b;
  la.items = w->items_long;
  la.ctr = w->ctr;
  la.subst = w->subst;
  la.asz = cs.asz;
  la.alpha = cs.alpha;
  la.beta = cs.beta;
  la.scores = P.scores;
  la.bnd = w->bnd_long;
  la.flags = w->flags;
  AS_HIP(launch_long_dp_i32(mode, la, long_dp_i32_blocks_per_cu(mode, cs.asz) * w->num_cu, stream));
  if (cs.allow16 || mode == kLocal) {  // saturated packed pairs (16-bit list or kVarP16)
    args.items = w->rerun;
    args.n_items = &w->ctr->n_rerun32;
    args.next = &w->ctr->next_rerun32;
    args.bnd_rows = P.bnd_rows;   // kVarP16 re-runs may span several stripes
    const int grid_r = full_dp_i32_blocks_per_cu(mode, cs.asz, kmask_of_variant(kVarI32K16)) * w->num_cu;
    AS_HIP(launch_full_dp_i32(mode, args, kmask_of_variant(kVarI32K16), grid_r, stream));
  }
  AS_HIP(hipMemcpyAsync(w->host_ctr, w->ctr, kCountersHead, hipMemcpyDeviceToHost, stream));
  return AS_OK;
}

void destroy_plan(PlanImpl *P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  free_workspace(P->ws);
  delete P;
}

extern "C" int as_plan_create(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                              const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                              int32_t *scores_out, as_plan **plan_out, void *stream_ptr) {
  if (!scoring || !offs_a || !offs_b || !seqs_a || !seqs_b || !scores_out || !scoring->subst || !plan_out)
    return AS_ERR_NULL;
  *plan_out = nullptr;
  if (n_pairs < 1 || n_pairs >= ((int64_t)1 << 31) - 1) return AS_ERR_ARG;
  CallScoring cs;
  int rc = check_scoring(scoring, mode, &cs);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_ptr;
  int dev = 0;
  AS_HIP(hipGetDevice(&dev));
  PlanImpl *P = new PlanImpl();
  auto fail = [&](int code) {
    destroy_plan(P);
    return code;
  };
  if ((rc = init_workspace(P->ws, dev))) return fail(rc);
  Workspace *w = &P->ws;
  P->cs = cs;
  {
    std::lock_guard<std::mutex> guard(g_lock);
    P->rp = route_params(cs, n_pairs);
    P->rp.long16 = 0;  // plans keep the 32-bit wavefront
  }
  P->seqs_a = seqs_a;
  P->seqs_b = seqs_b;
  P->offs_a = offs_a;
  P->offs_b = offs_b;
  P->n_pairs = n_pairs;
  P->scores = scores_out;
  if ((rc = lists_capacity(w, n_pairs))) return fail(rc);
  if (hipMemcpyAsync(w->subst, scoring->subst, (size_t)cs.asz * cs.asz, hipMemcpyHostToDevice, stream) !=
      hipSuccess)
    return fail(AS_ERR_HIP);
  // planning run: classification and wavefront preparation, to size the buffers
  if (hipMemsetAsync(w->ctr, 0, sizeof(Counters), stream) != hipSuccess) return fail(AS_ERR_HIP);
  if ((rc = launch_classify(w, P->rp, offs_a, offs_b, nullptr, n_pairs, scores_out, stream))) return fail(rc);
  hipLaunchKernelGGL(long_prep_kernel, dim3(1), dim3(256), 0, stream, w->items_long, w->ctr,
                     long_dp_i32_stripe_width(cs.asz), mode, scores_out, (int64_t)0, (int64_t)0);
  if (hipGetLastError() != hipSuccess) return fail(AS_ERR_HIP);
  Counters c;
  if ((rc = read_counters(w, stream, &c))) return fail(rc);
  if ((rc = status_to_code(c.status))) return fail(rc);
  // the 32-bit kernel covers every K the table can route (contents may change between replays)
  int kmask = kmask_of_variant(kVarI32K16);
  for (int b = 0; b < kLenBins; ++b) {
    const int v = P->rp.var_of_bin[b];
    if (v == kVarI32K8 || v == kVarI32K16 || v == kVarI32K32) kmask |= kmask_of_variant(v);
  }
  P->kmask = kmask;
  P->bnd_rows = (int64_t)(c.max_rows_multi > 0 ? c.max_rows_multi : 0) + 1;
  const int grid32 = full_dp_i32_blocks_per_cu(mode, cs.asz, kmask) * w->num_cu;
  const int grid_r = full_dp_i32_blocks_per_cu(mode, cs.asz, kmask_of_variant(kVarI32K16)) * w->num_cu;
  const int64_t slots = (int64_t)(grid32 > grid_r ? grid32 : grid_r) * kGroupsPerWave;
  if ((rc = grow((void **)&w->bnd, &w->bnd_cap, slots * 2 * P->bnd_rows, sizeof(int2)))) return fail(rc);
  P->bnd_long_cap = c.long_bnd_total > 0 ? c.long_bnd_total : 1;
  P->flags_cap = c.n_long_tasks > 0 ? c.n_long_tasks : 1;
  if ((rc = grow((void **)&w->bnd_long, &w->bnd_long_cap, P->bnd_long_cap, sizeof(int2)))) return fail(rc);
  if ((rc = grow((void **)&w->flags, &w->flags_cap, P->flags_cap, sizeof(int32_t)))) return fail(rc);
  // capture on a private stream of default priority
  if (hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess) return fail(AS_ERR_HIP);
  if (hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(AS_ERR_HIP);
  rc = enqueue_plan(*P, P->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(P->cap_stream, &g);
  P->graph = g;
  if (rc) return fail(rc);
  if (ec != hipSuccess || !g) return fail(AS_ERR_HIP);
  if (hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess) return fail(AS_ERR_HIP);
  *plan_out = reinterpret_cast<as_plan *>(P);
  return AS_OK;
}

extern "C" int as_plan_run(as_plan *plan, void *stream_ptr) {
  if (!plan) return AS_ERR_NULL;
  PlanImpl *P = reinterpret_cast<PlanImpl *>(plan);
  hipStream_t stream = (hipStream_t)stream_ptr;
  AS_HIP(hipGraphLaunch(P->exec, stream));
  AS_HIP(hipStreamSynchronize(stream));
  const Counters *c = P->ws.host_ctr;
  return status_to_code(c->status);
}

extern "C" int as_plan_destroy(as_plan *plan) {
  destroy_plan(reinterpret_cast<PlanImpl *>(plan));
  return AS_OK;
}

extern "C" int as_set_variants(int32_t mode, const int8_t *table) {
  if (mode < 0 || mode > 2) return AS_ERR_ARG;
  if (table)
    for (int b = 0; b < kLenBins; ++b)
      if (table[b] < -1 || table[b] >= kNumVariants) return AS_ERR_ARG;
  std::lock_guard<std::mutex> guard(g_lock);
  for (int b = 0; b < kLenBins; ++b) g_variants[mode][b] = table ? table[b] : (int8_t)-1;
  return AS_OK;
}

extern "C" int as_get_variants(int32_t mode, int8_t *table_out) {
  if (!table_out) return AS_ERR_NULL;
  if (mode < 0 || mode > 2) return AS_ERR_ARG;
  std::lock_guard<std::mutex> guard(g_lock);
  for (int b = 0; b < kLenBins; ++b) table_out[b] = g_variants[mode][b];
  return AS_OK;
}

extern "C" int as_autotune(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                           const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                           int32_t sample_pairs, float *gcups_out, int8_t *table_out, void *stream_ptr) {
  if (!scoring || !offs_a || !offs_b || !seqs_a || !seqs_b || !scoring->subst) return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1 || sample_pairs < 1) return AS_ERR_ARG;
  CallScoring cs;
  int rc = check_scoring(scoring, mode, &cs);
  if (rc) return rc;
  if (gcups_out)
    for (int i = 0; i < kLenBins * kNumVariants; ++i) gcups_out[i] = 0.f;
  std::lock_guard<std::mutex> guard(g_lock);
  Workspace *w = nullptr;
  if ((rc = get_workspace(&w))) return rc;
  hipStream_t stream = (hipStream_t)stream_ptr;
  if (n_pairs > 0) {
    if ((rc = lists_capacity(w, n_pairs))) return rc;
    if ((rc = grow((void **)&w->tune_scores, &w->tune_scores_cap, n_pairs, sizeof(int32_t)))) return rc;
    AS_HIP(hipMemcpyAsync(w->subst, scoring->subst, (size_t)cs.asz * cs.asz, hipMemcpyHostToDevice, stream));
    // pairs and cells per length bin under the automatic rule
    RouteParams rp = route_params(cs, n_pairs);
    for (int b = 0; b < kLenBins; ++b) rp.var_of_bin[b] = -1;
    AS_HIP(hipMemsetAsync(w->ctr, 0, sizeof(Counters), stream));
    if ((rc = launch_classify(w, rp, offs_a, offs_b, nullptr, n_pairs, w->tune_scores, stream))) return rc;
    Counters c0;
    if ((rc = read_counters(w, stream, &c0))) return rc;
    if ((rc = status_to_code(c0.status))) return rc;
    const bool timing_was = g_timing;
    g_timing = true;
    // A sample of a bin: every stride-th pair, at most sample_pairs pairs
    // and about 1e11 cells (tens of milliseconds per variant).
    const double cell_cap = 1e11;
    int32_t strides[kLenBins] = {};  // each measured bin's sample stride (0: no pairs)
    for (int b = 0; b < kLenBins; ++b) {
      int64_t cnt = 0;
      for (int l = 0; l < kLists; ++l) cnt += c0.bin_count[l][b];
      if (cnt == 0) continue;
      int64_t stride = cnt / sample_pairs;
      const int64_t by_cells = (int64_t)((double)c0.bin_cells[b] / cell_cap);
      if (by_cells > stride) stride = by_cells;
      if (stride < 1) stride = 1;
      float best_g = -1.f;
      int best_v = -1;
      for (int v = 0; v < kNumVariants; ++v) {
        if (v == kVarI16 && !cs.allow16) continue;
        if (v == kVarP16 && !rp.allowP16) continue;
        if (v == kVarLong && ((int64_t)64 << b) <= long_dp_i32_stripe_width(cs.asz)) continue;
        RouteParams t = rp;
        t.only_bin = b;
        t.var_of_bin[b] = (int8_t)v;
        t.sample_stride[b] = (int32_t)(stride > (1 << 30) ? (1 << 30) : stride);
        float ms_best = -1.f;
        double cells = 0;
        for (int rep = 0; rep < 2; ++rep) {
          AS_HIP(hipMemsetAsync(w->ctr, 0, sizeof(Counters), stream));
          if ((rc = launch_classify(w, t, offs_a, offs_b, nullptr, n_pairs, w->tune_scores, stream))) break;
          Counters c;
          if ((rc = read_counters(w, stream, &c))) break;
          memset(&g_last_timing, 0, sizeof(g_last_timing));
          if ((rc = run_full_lists(w, cs, seqs_a, seqs_b, w->tune_scores, stream, true, c))) break;
          const float ms = g_last_timing.full16_ms + g_last_timing.full32_ms + g_last_timing.long_ms +
                           g_last_timing.long16_ms + g_last_timing.rerun32_ms;
          cells = (double)(c.route_cells[kList16] + c.route_cells[kList32] + c.route_cells[kListLong] +
                           c.route_cells[kListLong16]);
          if (ms_best < 0.f || ms < ms_best) ms_best = ms;
        }
        if (rc) break;
        const float g = ms_best > 0.f ? (float)(cells / (ms_best * 1e-3) / 1e9) : 0.f;
        if (gcups_out) gcups_out[b * kNumVariants + v] = g;
        if (g > best_g) {
          best_g = g;
          best_v = v;
        }
      }
      if (rc) break;
      g_variants[mode][b] = (int8_t)best_v;
      strides[b] = (int32_t)(stride > (1 << 30) ? (1 << 30) : stride);
    }
    // Precision: where the scoring admits FP16 cells and the tuned table
    // sends a bin to the packed kernel, time the sampled bins under both
    // cell types (pairs an FP16 range bound refuses take the 32-bit kernels,
    // which the timing includes) and keep the faster for the automatic
    // setting.
    bool packed_bin = false;
    for (int b = 0; b < kLenBins; ++b)
      packed_bin = packed_bin || (strides[b] > 0 && (g_variants[mode][b] == kVarI16 ||
                                                     (g_variants[mode][b] < 0 && cs.allow16)));
    if (!rc && cs.half_adm != kCellI16 && packed_bin) {
      float ms_of[2] = {-1.f, -1.f};
      for (int h = 0; h < 2 && !rc; ++h) {
        CallScoring ch = cs;
        ch.half = h ? cs.half_adm : kCellI16;
        RouteParams t = route_params(ch, n_pairs);
        for (int b = 0; b < kLenBins; ++b) {
          t.var_of_bin[b] = g_variants[mode][b];
          t.sample_stride[b] = strides[b] > 0 ? strides[b] : (1 << 30);
        }
        for (int rep = 0; rep < 2; ++rep) {
          AS_HIP(hipMemsetAsync(w->ctr, 0, sizeof(Counters), stream));
          if ((rc = launch_classify(w, t, offs_a, offs_b, nullptr, n_pairs, w->tune_scores, stream))) break;
          Counters c;
          if ((rc = read_counters(w, stream, &c))) break;
          memset(&g_last_timing, 0, sizeof(g_last_timing));
          if ((rc = run_full_lists(w, ch, seqs_a, seqs_b, w->tune_scores, stream, true, c))) break;
          const float ms = g_last_timing.full16_ms + g_last_timing.full32_ms + g_last_timing.long_ms +
                           g_last_timing.long16_ms + g_last_timing.rerun32_ms;
          if (ms_of[h] < 0.f || ms < ms_of[h]) ms_of[h] = ms;
        }
      }
      if (!rc) g_half_pref[mode] = (int8_t)(ms_of[1] < ms_of[0] ? 1 : 0);
    }
    g_timing = timing_was;
    if (rc) return rc;
  }
  if (table_out)
    for (int b = 0; b < kLenBins; ++b) table_out[b] = g_variants[mode][b];
  return AS_OK;
}

extern "C" const char *as_strerror(int code) {
  switch (code) {
    case AS_OK: return "success";
    case AS_ERR_NULL: return "a required pointer is NULL";
    case AS_ERR_OFFSETS: return "offsets decrease or are negative";
    case AS_ERR_RESIDUE: return "a residue code is >= alphabet_size";
    case AS_ERR_SCORING: return "invalid scoring (alphabet size, alpha, beta, mode or sigma range)";
    case AS_ERR_RANGE: return "a score could leave the 32-bit range";
    case AS_ERR_HIP: return "a HIP runtime call failed or a device-side wait stalled";
    case AS_ERR_ARG: return "an argument is out of range";
    case AS_ERR_SCRATCH: return "the batch needs more scratch than the no-allocation entry point's static array";
    default: return "unknown error";
  }
}

extern "C" int as_release_workspace(void) {
  release_learned_workspace();  // takes its own lock, never while holding this one
  release_traceback_workspace();
  std::lock_guard<std::mutex> guard(g_lock);
  for (Workspace &w : g_ws) {
    if (w.device < 0) continue;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(w.device);
    free_workspace(w);
    (void)hipSetDevice(cur);
  }
  return AS_OK;
}

extern "C" int as_set_band_packing(int32_t on) {
  std::lock_guard<std::mutex> guard(g_lock);
  const int prev = g_band16 ? 1 : 0;
  g_band16 = on != 0;
  return prev;
}

extern "C" int as_set_half_cells(int mode) {
  std::lock_guard<std::mutex> guard(g_lock);
  const int prev = g_half_cells;
  g_half_cells = (mode == 0 || mode == 1) ? mode : 2;
  return prev;
}

extern "C" int as_half_cells_preference(int32_t mode, int32_t pref, int32_t set) {
  if (mode < 0 || mode > 2) return AS_ERR_ARG;
  if (set && (pref < -1 || pref > 1)) return AS_ERR_ARG;
  std::lock_guard<std::mutex> guard(g_lock);
  const int prev = g_half_pref[mode];
  if (set) g_half_pref[mode] = (int8_t)pref;
  return prev;
}

extern "C" int as_set_i16_limit(int32_t limit) {
  std::lock_guard<std::mutex> guard(g_lock);
  const int32_t prev = g_i16_limit;
  g_i16_limit = (limit <= 0 || limit > 32767) ? 32767 : limit;
  return prev;
}

extern "C" int as_enable_timing(int on) {
  std::lock_guard<std::mutex> guard(g_lock);
  const int prev = g_timing ? 1 : 0;
  g_timing = on != 0;
  return prev;
}

extern "C" int as_last_timing(as_timing *out) {
  if (!out) return AS_ERR_NULL;
  std::lock_guard<std::mutex> guard(g_lock);
  *out = g_last_timing;
  return AS_OK;
}

extern "C" const char *as_build_info(void) {
  return "anyseq_mi gfx950: full DP int32 (16-lane DPP groups, K=16, int8 LDS profile); "
         "full DP packed int16x2 (2 pairs per group, K=16, v_perm register profile, alphabet <= 4); "
         "long-pair wavefront int32 (wave64 pipelines, 1024-column stripes); "
         "banded int32 (sheared band, K=4..64, v_perm scores, certificate + doubling)";
}
