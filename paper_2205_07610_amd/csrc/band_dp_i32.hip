// Banded Gotoh DP (global and semi-global), 32-bit cells, one 16-lane group
// per pair, with the acceptance test of the learned-band method.
//
// Sheared layout.  A band of diagonals lo <= j - i <= hi is a parallelogram;
// in sheared coordinates (i, k = j - i - lo) it is a rectangle of W = 16*K
// columns, and each lane owns K of them (lane t: k in [tK, tK+K)).  The
// recurrences of the paper's Eq. (1),(4),(5) become
//   diagonal H(i-1, j-1) -> (i-1, k)    : the same register, previous row
//   up       H/E(i-1, j) -> (i-1, k+1)  : the next register, previous row
//   left     H/F(i, j-1) -> (i, k-1)    : the previous register, same row
// Rows stream down the lanes exactly as in the full-matrix kernels (lane t
// computes row it + 1 - t in step it; F arrives from lane t-1 through DPP
// row_shr:1).  The one new dependency, "up" at a lane's last register, needs
// lane t+1's first register one row earlier -- which lane t+1 computes in the
// same step: every lane updates its first register first, the pair
// (E, H') of that register moves to lane t-1 with one DPP row_shl:1, and only
// then the remaining registers are updated.
//
// Scores.  sigma(q_i, s_j) + bias comes from one v_perm_b32 per four cells:
// the source bytes are the row residue's scores against the four letters
// (and padding bytes), the selector is a sliding window of the lane's column
// residue codes that shifts by one byte per row (v_alignbyte) and takes its
// new code from lane t+1 (or, at lane 15, from a feed).  The shifted frame
// X + beta*(i+j) of the full kernels is used, so a cell costs the same five
// operations; columns j <= 0 inside the band are padding columns whose
// scores reproduce the boundary column exactly (see full_dp_i16x2.hip).
//
// The band actually computed is [lo, lo + W - 1] with W the smallest lane
// width that holds the requested band, centred on it; it contains the
// requested band, so the acceptance bound computed for it is valid.
//
// Exact mode (EXACT = true) restricts the DP to the requested diagonals
// L <= j - i <= U themselves: a register whose diagonal lies outside is set
// to -infinity after every update (and at row 0), so no value crosses the
// band edge -- E only enters a cell from the diagonal above, F from the one
// below, and both come from masked registers there.  Columns j < 0 inside
// the band keep reproducing the boundary column along their own diagonal,
// which the mask never cuts.  The acceptance bound is then taken for [L, U].
// This mode produces the band labels (smallest accepted half-width).
#include "internal.h"

namespace asmi {
namespace {

// One-lane shifts inside a group of G lanes: a DPP row (G = 16) or the
// whole wave (G = 64); the first / last lane of the group keeps `old`.
template <int G>
__device__ __forceinline__ int shr1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, G == 16 ? 0x111 : 0x138, 0xF, 0xF, false);
}
template <int G>
__device__ __forceinline__ int shl1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, G == 16 ? 0x101 : 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ int imax3(int a, int b, int c) { return max(max(a, b), c); }
// Maximum over the lanes of a group.
template <int G>
__device__ __forceinline__ int group_max(int v) {
  if (G == 64) {
    v = max(v, __shfl_xor(v, 32));
    v = max(v, __shfl_xor(v, 16));
  }
  v = max(v, __shfl_xor(v, 8, 16));
  v = max(v, __shfl_xor(v, 4, 16));
  v = max(v, __shfl_xor(v, 2, 16));
  v = max(v, __shfl_xor(v, 1, 16));
  return v;
}
// Maximum over the groups of a wave of a value uniform inside each group.
template <int G>
__device__ __forceinline__ int wave_max_groups(int v) {
  if (G == 16) {
    v = max(v, __shfl_xor(v, 16));
    v = max(v, __shfl_xor(v, 32));
  }
  return v;
}

// Residue code of column j (1-based) for the v_perm selector: the residue
// itself, or 4 (a padding byte) outside 1..n.
__device__ __forceinline__ uint32_t col_code(const uint8_t *cols, int n, int j, int asz, int &bad) {
  if (j < 1 || j > n) return 4u;
  int c = cols[j - 1];
  if (c >= asz) { bad = 1; c = 0; }
  return (uint32_t)c;
}

template <int MODE, int K, bool EXACT, int G>
__global__ void __launch_bounds__(kWave) band_dp_i32_kernel(BandArgs a, int kc) {
  constexpr int W = G * K;
  constexpr int GPW = kWave / G;  // groups (pairs) per wave
  constexpr int NV = K / 4;  // selector words per lane
  const int lane = threadIdx.x;
  const int g = lane / G;
  const int t = lane % G;
  const int alpha = a.alpha, beta = a.beta, amb = alpha - beta;
  const int asz = a.asz;
  const int cur = a.round & 1;
  const int n_list = a.ctr->n_band[cur][kc];
  const BandItem *list = a.sorted + a.sorted_base[kc];
  // score words: byte c of qword[r] = sigma(r, c) + alpha + beta (shifted frame)
  // padding byte (selector 4..7): alpha - beta (global) / alpha + beta (semi)
  const uint32_t padword = (uint32_t)((MODE == kGlobal ? alpha - beta : alpha + beta) & 0xFF) * 0x01010101u;

  for (;;) {
    int base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr->next_band[kc], GPW);
    base = __shfl(base, 0);
    if (base >= n_list) break;
    const int item = base + g;
    const bool has = item < n_list;
    BandItem bi{};
    if (has) bi = list[item];
    const PairDesc &d = bi.d;
    const int m = has ? d.m : 0, n = d.n;
    const bool tr = (d.flags & kTransposed) != 0;
    const uint8_t *rows = (tr ? a.seqs_b : a.seqs_a) + d.row_off;
    const uint8_t *cols = (tr ? a.seqs_a : a.seqs_b) + d.col_off;
    // band limits (requested half-width bi.w, widened to W and centred)
    const int L = min(0, n - m) - bi.w;
    const int U = max(0, n - m) + bi.w;
    const int lo = L - (W - (U - L + 1)) / 2;
    const int hi = lo + W - 1;
    const int kb = t * K;
    // registers of this lane inside [L, U] (exact mode)
    const int xa = L - lo - kb, xb = U - lo - kb;
    auto outside = [&](int x) -> bool { return EXACT && (x < xa || x > xb); };
    int bad = 0;

    // ---- state at row 0 (and the sheared column codes of row -t) ----
    // Every lane updates its registers in every step; a lane whose row has not
    // started yet (row <= 0) is reset to these row-0 values afterwards, and a
    // lane's results are taken when its row reaches m.  No step is masked.
    auto init_h = [&](int x) -> int {
      const int j = lo + kb + x;  // column of register x at row 0
      if (outside(x)) return kNegInf32;
      if (MODE == kGlobal) return (j == 0) ? beta - alpha : 2 * beta - 2 * alpha;
      return beta * j + beta - alpha;
    };
    int Ha[K], Ee[K], D[K];
#pragma unroll
    for (int x = 0; x < K; ++x) {
      Ha[x] = init_h(x);
      Ee[x] = kNegInf32;
      D[x] = kNegInf32;
    }
    uint32_t win[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uint32_t w = 0;
      for (int b = 0; b < 4; ++b)
        w |= col_code(cols, n, -t + lo + kb + 4 * v + b, asz, bad) << (8 * b);
      win[v] = w;
    }
    int fout = kNegInf32;
    uint32_t qrow = 0;
    int rowoff = beta * (1 - t);
    int res = kNegInf32;   // this lane's candidate for the banded score
    const int kn = n - m - lo;  // register index of column n at row m

    const int its = m > 0 ? m + G - 1 : 0;
    const int its_max = wave_max_groups<G>(its);
    // feeds, 16 steps per refill: row score words travel down from lane 0
    // (row_shr), new column codes enter at lane 15 (element u in lane 15-u)
    auto qword = [&](int idx) -> uint32_t {
      if (idx < 0 || idx >= m) return 0u;
      int r = rows[idx];
      if (r >= asz) { bad = 1; r = 0; }
      return a.qwords[(tr ? 32 : 0) + r];
    };
    uint32_t qfeed = qword(t);
    // new column codes enter at the group's last lane: element u of a chunk
    // sits in lane G-1-u (the last 16 lanes)
    uint32_t cfeed = col_code(cols, n, (G - 1 - t) - (G - 2) + lo + W - 1, asz, bad);
    for (int it0 = 0; it0 < its_max; it0 += kGroup) {
      const uint32_t qnext = qword(it0 + kGroup + t);
      const uint32_t cnext = col_code(cols, n, it0 + kGroup + (G - 1 - t) - (G - 2) + lo + W - 1, asz, bad);
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int row = it0 + u + 1 - t;
        // advance this lane's column window to `row`
        const uint32_t right = (uint32_t)shl1<G>((int)(cfeed << 8), (int)win[0]);  // byte 1 = new code
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const uint32_t nxt = (v + 1 < NV) ? win[v + 1] : (right >> 8);
          win[v] = __builtin_amdgcn_alignbyte(nxt, win[v], 1);
        }
        qrow = (uint32_t)shr1<G>((int)qfeed, (int)qrow);
        const int fl = shr1<G>(kNegInf32, fout);
        // phase A: diagonal sums and E from the previous row's registers
        int tt[K], ee[K];
#pragma unroll
        for (int x = 0; x < K; ++x) {
          const uint32_t sw = __builtin_amdgcn_perm(padword, qrow, win[x >> 2]);
          tt[x] = Ha[x] + (int)((sw >> (8 * (x & 3))) & 0xFF);
          if (x + 1 < K) ee[x] = max(Ee[x + 1], Ha[x + 1]);
        }
        // register 0, then its (E, H') to lane t-1 (one row above that lane's last register)
        int f = fl;
        {
          const int h = imax3(tt[0], K > 1 ? ee[0] : kNegInf32, f);
          Ha[0] = outside(0) ? kNegInf32 : h - amb;
          Ee[0] = K > 1 ? ee[0] : kNegInf32;
          f = max(f, Ha[0]);
          if (MODE == kSemiGlobal) D[0] = max(K > 1 ? D[1] : kNegInf32, Ha[0] - rowoff);
        }
        // pipeline fill (a uniform branch, taken in the first 16 steps only)
        const bool filling = __builtin_amdgcn_ballot_w64(row <= 0) != 0;
        if (filling && row <= 0) {
          Ha[0] = init_h(0);
          Ee[0] = kNegInf32;
          D[0] = kNegInf32;
        }
        const int eR = shl1<G>(kNegInf32, max(Ee[0], Ha[0]));
        const int dR = (MODE == kSemiGlobal) ? shl1<G>(kNegInf32, D[0]) : 0;
#pragma unroll
        for (int x = 1; x < K; ++x) {
          const int e = (x + 1 < K) ? ee[x] : eR;
          const int h = imax3(tt[x], e, f);
          Ha[x] = outside(x) ? kNegInf32 : h - amb;
          Ee[x] = e;
          f = max(f, Ha[x]);
          if (MODE == kSemiGlobal) D[x] = max((x + 1 < K) ? D[x + 1] : dR, Ha[x] - rowoff);
        }
        fout = f;
        if (filling && row <= 0) {  // pipeline fill: back to row 0
#pragma unroll
          for (int x = 1; x < K; ++x) {
            Ha[x] = init_h(x);
            Ee[x] = kNegInf32;
            D[x] = kNegInf32;
          }
          fout = kNegInf32;
        }
        if (__builtin_amdgcn_ballot_w64(row == m) != 0 && row == m) {
          // this lane's last row: take its part of the result
          if (MODE == kGlobal) {
            if (kn / K == t) {
#pragma unroll
              for (int x = 0; x < K; ++x)
                if (x == kn % K) res = Ha[x] + amb - beta * (m + n);
            }
          } else {
            // last row: H(m, j) = H'(m, j) + alpha - beta - beta*(m + j), columns 0..n
            int lr = kNegInf32;
#pragma unroll
            for (int x = 0; x < K; ++x) {
              const int j = m + lo + kb + x;
              if (j >= 0 && j <= n) lr = max(lr, Ha[x] - beta * j);
            }
            res = lr + amb - beta * m;
            // last column: D follows column n, at row m it sits in register kn
            if (kn / K == t) {
#pragma unroll
              for (int x = 0; x < K; ++x)
                if (x == kn % K) res = max(res, D[x] + amb - beta * n);
            }
          }
        }
        rowoff += beta;
        qfeed = (uint32_t)shl1<G>((int)qfeed, (int)qfeed);
        cfeed = (uint32_t)shr1<G>((int)cfeed, (int)cfeed);
      }
      qfeed = qnext;
      cfeed = cnext;
    }

    // ---- banded score ----
    int score = group_max<G>(res);
    // H(0, n) = 0 counts when that boundary cell lies in the band (H(m, 0) is
    // the last row's column 0, already among the registers when in the band)
    const int blo = EXACT ? L : lo, bhi = EXACT ? U : hi;  // the band scored
    if (MODE == kSemiGlobal && n <= bhi) score = max(0, score);
    if (bad) atomicOr(&a.ctr->status, kStatusBadResidue);
    if (!has || t != 0) continue;

    // ---- acceptance (certificate), next band or full-DP fallback ----
    const int lo_ab = tr ? -bhi : blo, hi_ab = tr ? -blo : bhi;  // limits in A/B orientation
    if (a.lo_out) { a.lo_out[d.pair] = lo_ab; a.hi_out[d.pair] = hi_ab; }
    int64_t ub = 0;
    const bool leave = band_leave_bound(m, n, blo, bhi, a.sigma_max, alpha, beta, MODE, &ub);
    const bool accept = !leave || (int64_t)score >= ub;
    if (a.raw) {
      a.scores[d.pair] = score;
      if (a.accept_out) a.accept_out[d.pair] = accept ? 1 : 0;
      continue;
    }
    atomicAdd(&a.ctr->band_cells, (unsigned long long)((long long)m * W));
    if (accept) {
      a.scores[d.pair] = score;
      atomicAdd(&a.ctr->band_accepted[a.round < kMaxBandRounds ? a.round : kMaxBandRounds - 1], 1);
      continue;
    }
    band_requeue(a, d, bi.w, MODE, W, score);
  }
}

// Lane-width classes: 64, 128, 192, 256 and 384 diagonals on 16-lane groups
// (K = 4, 8, 12, 16, 24; four pairs per wave), 512, 768, 1024, 1280 and 1536
// on whole waves (K = 8, 12, 16, 20, 24; one pair per wave), which keeps the
// registers a lane holds low enough for several waves per SIMD.
static_assert(kBandClasses == 10, "class table");
static_assert(sizeof(((Counters *)0)->next_band) == kBandClasses * sizeof(int32_t), "counters");
template <int MODE, bool EXACT>
hipError_t launch_mode(const BandArgs &args, int kc, int grid, hipStream_t stream) {
  switch (kc) {
    case 0: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 4, EXACT, 16>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    case 1: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 8, EXACT, 16>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    case 2: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 12, EXACT, 16>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    case 3: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 16, EXACT, 16>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    case 4: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 24, EXACT, 16>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    case 5: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 8, EXACT, 64>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    case 6: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 12, EXACT, 64>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    case 7: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 16, EXACT, 64>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    case 8: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 20, EXACT, 64>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
    default: hipLaunchKernelGGL((band_dp_i32_kernel<MODE, 24, EXACT, 64>), dim3(grid), dim3(kWave), 0, stream, args, kc); break;
  }
  return hipGetLastError();
}

template <int MODE, int K, int G>
int occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band_dp_i32_kernel<MODE, K, false, G>, kWave, 0) !=
          hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

}  // namespace

hipError_t launch_band_dp_i32(int mode, int kc, const BandArgs &args, int grid, hipStream_t stream) {
  if (args.exact)
    return mode == kGlobal ? launch_mode<kGlobal, true>(args, kc, grid, stream)
                           : launch_mode<kSemiGlobal, true>(args, kc, grid, stream);
  return mode == kGlobal ? launch_mode<kGlobal, false>(args, kc, grid, stream)
                         : launch_mode<kSemiGlobal, false>(args, kc, grid, stream);
}

int band_dp_i32_pairs_per_wave(int kc) { return kc >= 5 ? 1 : kGroupsPerWave; }

int band_dp_i32_blocks_per_cu(int mode, int kc) {
  if (mode == kGlobal) {
    switch (kc) {
      case 0: return occupancy<kGlobal, 4, 16>();
      case 1: return occupancy<kGlobal, 8, 16>();
      case 2: return occupancy<kGlobal, 12, 16>();
      case 3: return occupancy<kGlobal, 16, 16>();
      case 4: return occupancy<kGlobal, 24, 16>();
      case 5: return occupancy<kGlobal, 8, 64>();
      case 6: return occupancy<kGlobal, 12, 64>();
      case 7: return occupancy<kGlobal, 16, 64>();
      case 8: return occupancy<kGlobal, 20, 64>();
      default: return occupancy<kGlobal, 24, 64>();
    }
  }
  switch (kc) {
    case 0: return occupancy<kSemiGlobal, 4, 16>();
    case 1: return occupancy<kSemiGlobal, 8, 16>();
    case 2: return occupancy<kSemiGlobal, 12, 16>();
    case 3: return occupancy<kSemiGlobal, 16, 16>();
    case 4: return occupancy<kSemiGlobal, 24, 16>();
    case 5: return occupancy<kSemiGlobal, 8, 64>();
    case 6: return occupancy<kSemiGlobal, 12, 64>();
    case 7: return occupancy<kSemiGlobal, 16, 64>();
    case 8: return occupancy<kSemiGlobal, 20, 64>();
    default: return occupancy<kSemiGlobal, 24, 64>();
  }
}

}  // namespace asmi
