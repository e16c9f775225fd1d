// Full Gotoh DP with packed 16-bit cells: two alignments per 16-lane group,
// one in the low and one in the high half of every 32-bit register, so each
// packed VALU instruction updates two DP cells (the paper's section 3.2
// "two independent alignments in one register" idea, with exact int16
// arithmetic instead of half floats).
//
// Mapping, frames and per-cell recurrences are those of the 32-bit kernel
// (full_dp_i32.hip): lane t owns K adjacent columns, step `it` computes row
// it + 1 - t, the rightmost H/F of lane t-1 arrives through DPP row_shr:1,
// global and semi-global run in the shifted frame X + beta*(i+j) (no beta
// anywhere in the cell update), local in the plain frame with E and F
// clamped at 0.  Differences:
//
//  * Profile: the alphabet has at most 4 letters here, so each lane keeps,
//    per owned column and per half, one 32-bit word whose byte c holds
//    sigma(c, s_j) + bias.  One v_perm_b32 per cell pair selects the byte of
//    the current row's residue for each half and zero-extends both into a
//    packed pair -- no LDS traffic at all.  Row residues travel down the
//    lanes as the v_perm selector itself.
//  * Padding: every mode pads on the LEFT so that column n of both halves is
//    the last register of lane 15.  Local/semi-global padding columns score
//    0 (they reproduce the boundary column H = 0); global padding columns
//    use the profile value alpha - beta, which keeps the shifted frame flat
//    at its boundary value: in the shifted frame the global boundary
//    H(i,0) = -alpha - beta(i-1) is the constant beta - alpha.
//  * Rows past a half's own length use selector 0 (score -bias), which can
//    only lower cells; local and semi-global maxima are unaffected, global
//    results are snapshot at the half's last row.
//  * Range: global and semi-global pairs are queued here only when an a
//    priori bound keeps every shifted cell inside int16; local cells are
//    bounded below by -alpha and are added with signed saturation, so a
//    pair whose maximum reaches 32767 is re-queued for the 32-bit kernel.
//  * Half precision (the paper's own choice of packed type, selectable per
//    call): the same recurrences on pairs of FP16 values.  Profile bytes are
//    FP8 E4M3 codes of sigma + bias (exact for the integers 0..16), turned
//    into a pair of halves by one packed conversion after the v_perm; the
//    clamped local updates take a max with 0 instead of an unsigned
//    saturating subtract.  Integers are exact in FP16 up to 2048 in
//    magnitude: global and semi-global pairs come here only under a priori
//    bounds below that, and a local pair whose maximum reaches the
//    threshold (at most 2048 - 64, so every value before it was exact) is
//    re-run with 32 bits like a saturated int16 pair.
#include <type_traits>

#include "internal.h"

namespace asmi {
namespace {

constexpr int kK16 = 16;
constexpr int kK8 = 8;
constexpr int kK32 = 32;
constexpr int kW16 = kGroup * kK16;
constexpr short kNeg16 = -16384;

typedef short s2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int as_i(s2 v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ s2 as_s2(int v) { return __builtin_bit_cast(s2, v); }
__device__ __forceinline__ s2 pk(int lo, int hi) {
  s2 r;
  r.x = (short)lo;
  r.y = (short)hi;
  return r;
}
__device__ __forceinline__ s2 vmax(s2 a, s2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s2 sat_sub_u(s2 a, s2 b) {
  return __builtin_bit_cast(s2, __builtin_elementwise_sub_sat(__builtin_bit_cast(u2, a),
                                                              __builtin_bit_cast(u2, b)));
}
__device__ __forceinline__ int dpp_shr1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x111, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_shl1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x101, 0xF, 0xF, false);
}
__device__ __forceinline__ s2 group_max2(s2 v) {
  v = vmax(v, as_s2(__shfl_xor(as_i(v), 8, 16)));
  v = vmax(v, as_s2(__shfl_xor(as_i(v), 4, 16)));
  v = vmax(v, as_s2(__shfl_xor(as_i(v), 2, 16)));
  v = vmax(v, as_s2(__shfl_xor(as_i(v), 1, 16)));
  return v;
}
// Half-precision pairs (the paper's section 3.2 arithmetic: two alignments
// in one register of two FP16 values).  Cells hold integers; they stay exact
// while every value is within +-2048 (11 significant bits), which the
// routing proves a priori for every pair it gives this variant.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int as_i(h2 v) { return __builtin_bit_cast(int, v); }
// IEEE maximum (no NaN canonicalisation; two nested ones fuse into one
// v_pk_maximum3_f16)
__device__ __forceinline__ h2 vmax(h2 a, h2 b) { return __builtin_elementwise_maximum(a, b); }
template <typename V> __device__ __forceinline__ V as_v(int v) { return __builtin_bit_cast(V, v); }
template <typename V> __device__ __forceinline__ V pkv(int lo, int hi) {
  V r;
  r.x = lo;
  r.y = hi;
  return r;
}
__device__ __forceinline__ int toi(short v) { return v; }
__device__ __forceinline__ int toi(_Float16 v) { return (int)v; }
// max(a - b, 0) for a >= 0 (E and F of local cells, clamped at 0)
__device__ __forceinline__ s2 clamp_sub(s2 a, s2 b) { return sat_sub_u(a, b); }
__device__ __forceinline__ h2 clamp_sub(h2 a, h2 b) { return vmax(a - b, pkv<h2>(0, 0)); }
// diagonal sum of local cells: signed saturation detects overflow of int16
// cells; half cells are proven in range, so a plain add
__device__ __forceinline__ s2 add_diag(s2 a, s2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ h2 add_diag(h2 a, h2 b) { return a + b; }
__device__ __forceinline__ h2 group_max2(h2 v) {
  v = vmax(v, as_v<h2>(__shfl_xor(as_i(v), 8, 16)));
  v = vmax(v, as_v<h2>(__shfl_xor(as_i(v), 4, 16)));
  v = vmax(v, as_v<h2>(__shfl_xor(as_i(v), 2, 16)));
  v = vmax(v, as_v<h2>(__shfl_xor(as_i(v), 1, 16)));
  return v;
}

// Profile bytes by cell type (kCellI16, kCellF16E4M3, kCellF16E5M2).
template <int CELL>
__host__ __device__ inline uint32_t profile_byte(int v) {
  return CELL == kCellF16E4M3 ? fp8_e4m3(v) : (CELL == kCellF16E5M2 ? fp8_e5m2(v) : (uint32_t)(v & 0xFF));
}

// Scores of a cell pair from the two halves' profile words and the
// selector.  int16: v_perm_b32 zero-extends the two selected bytes into the
// 16-bit halves.  E5M2: v_perm puts each byte in the upper byte of its half
// (lower byte zero), which is the FP16 value.  E4M3: v_perm puts the bytes
// in bytes 0 and 1 and one packed conversion makes two halves of them.
// v_perm selector for the row residues of both halves: it picks letter c0
// of the low half's word (source bytes 0..3) and letter c1 of the high
// half's word (source bytes 4..7) into the byte positions the cell type
// needs, every other byte zero.  A residue code of 12 ("no row") selects
// the constant 0 byte.
template <int CELL>
__device__ __forceinline__ uint32_t make_sel(int c0, int c1) {
  const uint32_t s0 = (c0 == 12) ? 0x0Cu : (uint32_t)c0;
  const uint32_t s1 = (c1 == 12) ? 0x0Cu : (uint32_t)(4 + c1);
  if (CELL == kCellF16E4M3) return s0 | (s1 << 8) | 0x0C0C0000u;
  if (CELL == kCellF16E5M2) return 0x0Cu | (s0 << 8) | 0x0C0000u | (s1 << 24);
  return s0 | 0x0C00u | (s1 << 16) | 0x0C000000u;
}
template <int CELL, typename V>
__device__ __forceinline__ V profile_pair(uint32_t phi, uint32_t plo, uint32_t sel) {
  const int b = (int)__builtin_amdgcn_perm(phi, plo, sel);
  if constexpr (CELL == kCellF16E4M3) return __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(b, 1.0f, false);
  else return as_v<V>(b);
}

__device__ __forceinline__ int wave_max_groups(int v) {
  v = max(v, __shfl_xor(v, 16));
  v = max(v, __shfl_xor(v, 32));
  return v;
}

// Profile word of column j: byte c = sigma(c, s_j) + bias for the row
// letters c, from the per-orientation table ptab (one word per column
// letter); padding columns hold pad_val in every byte.
__device__ __forceinline__ uint32_t profile_word(const uint32_t *ptab, const uint8_t *cols, int n, bool tr,
                                                 int j, int asz, uint32_t pad_word, int &bad) {
  if (j < 1 || j > n) return pad_word;
  int s = cols[j - 1];
  if (s >= asz) { bad = 1; s = 0; }
  return ptab[(tr ? 4 : 0) + s];
}

// The DP of one group's two pairs (low and high halves) once the register
// profiles are built: rows0/rows1 hold m0/m1 row residues, the halves have
// n0/n1 columns padded on the left to one stripe.  Returns both results, and
// for local mode whether a half reached the saturation limit.
template <int MODE, int K, int CELL = kCellI16>
__device__ __forceinline__ void duo_core(const uint8_t *rows0, const uint8_t *rows1, int m0, int m1, int n0,
                                         int n1, const uint32_t (&Plo)[K], const uint32_t (&Phi)[K], int asz,
                                         int alpha, int beta, int sat_limit, int lane, int &bad, int &r0,
                                         int &r1, bool &over0, bool &over1) {
  constexpr int W = kGroup * K;
  using V = typename std::conditional<CELL != kCellI16, h2, s2>::type;
  const int t = lane & 15;
  const int amb = alpha - beta;
  const V beta2 = pkv<V>(beta, beta);
  const V alpha2 = pkv<V>(alpha, alpha);
  const V amb2 = pkv<V>(amb, amb);
  const int P0 = W - n0, P1 = W - n1;     // left padding of each half
  const int mmax = max(m0, m1);
  const int msmall = min(m0, m1);
  const bool unequal = m0 != m1;
  const int its = mmax > 0 ? mmax + kGroup - 1 : 0;
  const int its_max = wave_max_groups(its);
  // ---- row-0 state ----
  V Ha[K], Ee[K];
#pragma unroll
  for (int x = 0; x < K; ++x) {
    const int j0 = t * K + x + 1 - P0, j1 = t * K + x + 1 - P1;
    if (MODE == kGlobal) {
      Ha[x] = pkv<V>(j0 == 0 ? beta - alpha : 2 * beta - 2 * alpha,
                 j1 == 0 ? beta - alpha : 2 * beta - 2 * alpha);
      Ee[x] = pkv<V>(kNeg16, kNeg16);
    } else if (MODE == kSemiGlobal) {
      Ha[x] = pkv<V>(beta * j0 + beta - alpha, beta * j1 + beta - alpha);
      Ee[x] = pkv<V>(kNeg16, kNeg16);
    } else {
      Ha[x] = pkv<V>(-alpha, -alpha);
      Ee[x] = pkv<V>(0, 0);   // E'(1, j) = max(E(1,j), 0) = 0
    }
  }
  V hl_prev;
  {
    const int j0 = t * K - P0, j1 = t * K - P1;
    if (MODE == kGlobal)
      hl_prev = pkv<V>(j0 == 0 ? beta - alpha : 2 * beta - 2 * alpha,
                   j1 == 0 ? beta - alpha : 2 * beta - 2 * alpha);
    else if (MODE == kSemiGlobal)
      hl_prev = pkv<V>(beta * j0 + beta - alpha, beta * j1 + beta - alpha);
    else
      hl_prev = pkv<V>(-alpha, -alpha);
  }
  int fout = (MODE == kLocal) ? 0 : as_i(pkv<V>(kNeg16, kNeg16));
  // left feed for lane 0 (row 1 first)
  V hb, fb;
  if (MODE == kGlobal) { hb = pkv<V>(2 * beta - 2 * alpha, 2 * beta - 2 * alpha); fb = hb; }
  else if (MODE == kSemiGlobal) {
    hb = pkv<V>(beta * (1 - P0) + beta - alpha, beta * (1 - P1) + beta - alpha);
    fb = hb;
  } else { hb = pkv<V>(-alpha, -alpha); fb = pkv<V>(0, 0); }
  V rowoff = pkv<V>(beta * (1 - t), beta * (1 - t));
  V rm = pkv<V>(0, 0);                       // local: running max of H
  V cm = pkv<V>(kNeg16, kNeg16);             // semi-global: max of H'(i,n) - beta*i
  V snap = pkv<V>(kNeg16, kNeg16);           // value of the shorter half at its last row

  auto load_sel = [&](int idx) -> int {
    int c0 = 12, c1 = 12;
    if (idx < m0) { c0 = rows0[idx]; if (c0 >= asz) { bad = 1; c0 = 0; } }
    if (idx < m1) { c1 = rows1[idx]; if (c1 >= asz) { bad = 1; c1 = 0; } }
    return (int)make_sel<CELL>(c0, c1);
  };
  int selfeed = load_sel(t);
  int sel = (int)make_sel<CELL>(12, 12);

  for (int it0 = 0; it0 < its_max; it0 += kGroup) {
    const int selnext = load_sel(it0 + kGroup + t);
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int row = it0 + u + 1 - t;
      sel = dpp_shr1(selfeed, sel);
      const V hl = as_v<V>(dpp_shr1(as_i(hb), as_i(Ha[K - 1])));
      const V fl = as_v<V>(dpp_shr1(as_i(fb), fout));
      if ((unsigned)(row - 1) < (unsigned)mmax) {
        // Phase A, independent per column: diagonal sums from the previous
        // row's values (and, shifted frame, E), so that phase B can overwrite
        // every state register in place.
        V tt[K];
#pragma unroll
        for (int x = 0; x < K; ++x) {
          const V p = profile_pair<CELL, V>(Phi[x], Plo[x], (uint32_t)sel);
          const V dg = (x == 0) ? hl_prev : Ha[x - 1];
          if (MODE == kLocal) {
            tt[x] = add_diag(dg, p);
          } else {
            tt[x] = dg + p;
            Ee[x] = vmax(Ee[x], Ha[x]);
          }
        }
        // Phase B, the F chain along the row.
        V f = fl;
#pragma unroll
        for (int x = 0; x < K; ++x) {
          if (MODE == kLocal) {
            const V h = vmax(vmax(tt[x], Ee[x]), f);
            rm = vmax(rm, h);
            Ha[x] = h - alpha2;
            Ee[x] = vmax(clamp_sub(Ee[x], beta2), Ha[x]);
            f = vmax(clamp_sub(f, beta2), Ha[x]);
          } else {
            const V h = vmax(vmax(tt[x], Ee[x]), f);
            Ha[x] = h - amb2;
            f = vmax(f, Ha[x]);
          }
        }
        fout = as_i(f);
        if (MODE == kSemiGlobal) cm = vmax(cm, Ha[K - 1] - rowoff);
        if (MODE != kLocal && unequal && row == msmall) {
          if (MODE == kGlobal) {
            if (t == kGroup - 1) snap = Ha[K - 1];
          } else {
            V lr = pkv<V>(kNeg16, kNeg16);
#pragma unroll
            for (int x = 0; x < K; ++x) {
              const int jp = t * K + x + 1;
              lr = vmax(lr, Ha[x] - pkv<V>(beta * (jp - P0), beta * (jp - P1)));
            }
            snap = lr;
          }
        }
      }
      hl_prev = hl;
      if (MODE == kSemiGlobal) {
        hb = hb + beta2;
        fb = hb;
      }
      rowoff = rowoff + beta2;
      selfeed = dpp_shl1(selfeed, selfeed);
    }
    selfeed = selnext;
  }

  // ---- results of both halves ----
  r0 = 0;
  r1 = 0;
  over0 = false;
  over1 = false;
  if (MODE == kLocal) {
    const V gm = group_max2(rm);
    r0 = toi(gm.x);
    r1 = toi(gm.y);
    over0 = r0 >= sat_limit;
    over1 = r1 >= sat_limit;
  } else if (MODE == kGlobal) {
    // lane 15, register K-1 holds column n of both halves
    const int src = (lane & ~(kGroup - 1)) + kGroup - 1;
    const V fin = as_v<V>(__shfl(as_i(Ha[K - 1]), src));
    const V sn = as_v<V>(__shfl(as_i(snap), src));
    const int v0 = toi((unequal && m0 < m1) ? sn.x : fin.x);
    const int v1 = toi((unequal && m1 < m0) ? sn.y : fin.y);
    r0 = v0 + amb - beta * (m0 + n0);
    r1 = v1 + amb - beta * (m1 + n1);
  } else {
    V lr = pkv<V>(kNeg16, kNeg16);
#pragma unroll
    for (int x = 0; x < K; ++x) {
      const int jp = t * K + x + 1;
      lr = vmax(lr, Ha[x] - pkv<V>(beta * (jp - P0), beta * (jp - P1)));
    }
    if (unequal) {
      if (m0 < m1) lr.x = snap.x;
      else lr.y = snap.y;
    }
    const V gl = group_max2(lr);
    const int src = (lane & ~(kGroup - 1)) + kGroup - 1;
    const V gc = as_v<V>(__shfl(as_i(cm), src));
    r0 = max(0, max(toi(gl.x) + amb - beta * m0, toi(gc.x) + amb - beta * n0));
    r1 = max(0, max(toi(gl.y) + amb - beta * m1, toi(gc.y) + amb - beta * n1));
  }
}

template <int MODE, int K, int CELL>
__global__ void __launch_bounds__(kWave) full_dp_i16_kernel(FullDp16Args a) {
  constexpr int W = kGroup * K;
  const int lane = threadIdx.x;
  const int g = lane >> 4;
  const int t = lane & 15;
  const int n_list = a.ctr->n_full16;
  const int alpha = a.alpha, beta = a.beta;
  const int asz = a.asz;
  const int bias = (MODE == kLocal) ? alpha : alpha + beta;
  const int pad_val = (MODE == kLocal) ? alpha : (MODE == kGlobal ? alpha - beta : alpha + beta);
  // int16: sigma + bias as an unsigned byte; FP16: its FP8 E4M3 code (the
  // routing admits the FP16 cells only when every such value is in 0..16)
  const uint32_t pad_word = profile_byte<CELL>(pad_val) * 0x01010101u;
  // profile words by (orientation, column letter): at most 4 letters here
  __shared__ uint32_t ptab[8];
  if (lane < 8) {
    const int o = lane >> 2, sl = lane & 3;
    uint32_t w = 0;
    if (sl < asz)
      for (int c = 0; c < asz; ++c) {
        const int sv = o ? a.subst[sl * asz + c] : a.subst[c * asz + sl];
        w |= profile_byte<CELL>(sv + bias) << (8 * c);
      }
    ptab[lane] = w;
  }
  __syncthreads();

  for (;;) {
    int base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr->next_full16, 2 * kGroupsPerWave);
    base = __shfl(base, 0);
    if (base >= n_list) break;
    const int i0 = base + 2 * g, i1 = i0 + 1;
    const bool has0 = i0 < n_list, has1 = i1 < n_list;
    PairDesc d0{0, 0, 0, 0, -1, 0}, d1{0, 0, 0, 0, -1, 0};
    if (has0) d0 = a.items[i0];
    if (has1) d1 = a.items[i1];
    const int m0 = d0.m, m1 = d1.m, n0 = d0.n, n1 = d1.n;
    const int P0 = W - n0, P1 = W - n1;     // left padding of each half
    const bool tr0 = (d0.flags & kTransposed) != 0, tr1 = (d1.flags & kTransposed) != 0;
    const uint8_t *rows0 = (tr0 ? a.seqs_b : a.seqs_a) + d0.row_off;
    const uint8_t *cols0 = (tr0 ? a.seqs_a : a.seqs_b) + d0.col_off;
    const uint8_t *rows1 = (tr1 ? a.seqs_b : a.seqs_a) + d1.row_off;
    const uint8_t *cols1 = (tr1 ? a.seqs_a : a.seqs_b) + d1.col_off;
    int bad = 0;

    // ---- register profile (paper: init_profile), both halves ----
    uint32_t Plo[K], Phi[K];
#pragma unroll
    for (int x = 0; x < K; ++x) {
      const int jp = t * K + x + 1;
      Plo[x] = profile_word(ptab, cols0, n0, tr0, jp - P0, asz, pad_word, bad);
      Phi[x] = profile_word(ptab, cols1, n1, tr1, jp - P1, asz, pad_word, bad);
    }

    int r0, r1;
    bool over0, over1;
    duo_core<MODE, K, CELL>(rows0, rows1, m0, m1, n0, n1, Plo, Phi, asz, alpha, beta, a.sat_limit, lane, bad,
                           r0, r1, over0, over1);
    if (bad) atomicOr(&a.ctr->status, kStatusBadResidue);
    if (t == 0) {
      if (has0) {
        if (over0) a.rerun[atomicAdd(&a.ctr->n_rerun32, 1)] = d0;
        else a.scores[d0.pair] = r0;
      }
      if (has1) {
        if (over1) a.rerun[atomicAdd(&a.ctr->n_rerun32, 1)] = d1;
        else a.scores[d1.pair] = r1;
      }
    }
  }
}

// All against all (the paper's evaluation workload: every read of a set
// against every other): the pairs are implicit, pair (q, s) is row sequence
// q against column sequence s, and its score goes to scores[q * ld + s] (or
// scores[s * ld + q] when the caller's roles are transposed).  A wave takes
// one column sequence of at most one packed stripe and a block of row
// sequences; it builds the column's register profile once and keeps it for
// the whole block, eight row sequences at a time (two per group, one per
// 16-bit half, both halves against the same column profile).  Local pairs
// that saturate are appended to the re-run list as descriptors for the
// 32-bit kernel.
// Global mode, every row sequence of length m: a group's row sequences run
// through its 16-lane pipeline back to back instead of one duo at a time,
// so the pipeline fills and drains once per group and block, not once per
// duo (16 steps of every m + 15).  The low halves take the group's queries
// q0(k) = first + 8k, the high halves q0(k) + 1; virtual row v of a half is
// row v - k m of its query k.  A lane that reaches the first row of a query
// puts its registers (and its diagonal input) back to the row-0 values; its
// left neighbour, one step ahead, already works on that query, and lane 0's
// boundary column is the same for every query in global mode.  Lane 15
// holds H'(m, n) of both halves when it finishes a query's last row.
template <int K, int CELL>
__device__ __forceinline__ void stream_global(const AllVsAllArgs &a, const uint32_t (&P)[K], int c, int n,
                                              int r_begin, int r_end, int lane, int &bad) {
  constexpr int W = kGroup * K;
  using V = typename std::conditional<CELL != kCellI16, h2, s2>::type;
  const int t = lane & 15, g = lane >> 4;
  const int alpha = a.alpha, beta = a.beta, amb = alpha - beta, asz = a.asz;
  const int m = a.eq_rows;
  const V amb2 = pkv<V>(amb, amb);
  const int pad = W - n;  // left padding of both halves
  const int first = r_begin + 2 * g;
  const int nk = first < r_end ? (r_end - first + 2 * kGroupsPerWave - 1) / (2 * kGroupsPerWave) : 0;
  const int total = nk * m;  // virtual rows of the group's low half
  const int its = nk > 0 ? total + kGroup - 1 : 0;
  const int its_max = wave_max_groups(its);
  const int neg_i = as_i(pkv<V>(kNeg16, kNeg16));
  auto row0 = [&](int j) -> int { return j == 0 ? beta - alpha : 2 * beta - 2 * alpha; };
  V Ha[K], Ee[K];
#pragma unroll
  for (int x = 0; x < K; ++x) {
    const int v0 = row0(t * K + x + 1 - pad);
    Ha[x] = pkv<V>(v0, v0);
    Ee[x] = as_v<V>(neg_i);
  }
  const int hl0 = row0(t * K - pad);
  V hl_prev = pkv<V>(hl0, hl0);
  int fout = neg_i;
  const V hb = pkv<V>(2 * beta - 2 * alpha, 2 * beta - 2 * alpha);
  // row letters of virtual row idx (0-based) of both halves; past a half's
  // queries the null letter (score 0), which never reaches a result
  auto load_sel = [&](int idx) -> int {
    int c0 = 12, c1 = 12;
    if (idx < total) {
      const int k = idx / m, loc = idx - k * m;
      const int q0 = first + 2 * kGroupsPerWave * k, q1 = q0 + 1;
      if (q0 < r_end) { c0 = a.seqs_r[a.offs_r[q0] + loc]; if (c0 >= asz) { bad = 1; c0 = 0; } }
      if (q1 < r_end) { c1 = a.seqs_r[a.offs_r[q1] + loc]; if (c1 >= asz) { bad = 1; c1 = 0; } }
    }
    return (int)make_sel<CELL>(c0, c1);
  };
  int selfeed = load_sel(t);
  int sel = (int)make_sel<CELL>(12, 12);
  int lrow = 0, kq = -1;  // this lane's row within its current query, and that query
  for (int it0 = 0; it0 < its_max; it0 += kGroup) {
    const int selnext = load_sel(it0 + kGroup + t);
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int row = it0 + u + 1 - t;
      sel = dpp_shr1(selfeed, sel);
      const V hl = as_v<V>(dpp_shr1(as_i(hb), as_i(Ha[K - 1])));
      const V fl = as_v<V>(dpp_shr1(as_i(hb), fout));
      if ((unsigned)(row - 1) < (unsigned)total) {
        if (lrow == m || lrow == 0) {  // the first row of the next query
          lrow = 0;
          ++kq;
#pragma unroll
          for (int x = 0; x < K; ++x) {
            const int v0 = row0(t * K + x + 1 - pad);
            Ha[x] = pkv<V>(v0, v0);
            Ee[x] = as_v<V>(neg_i);
          }
          hl_prev = pkv<V>(hl0, hl0);
        }
        ++lrow;
        V tt[K];
#pragma unroll
        for (int x = 0; x < K; ++x) {
          const V p = profile_pair<CELL, V>(P[x], P[x], (uint32_t)sel);
          const V dg = (x == 0) ? hl_prev : Ha[x - 1];
          tt[x] = dg + p;
          Ee[x] = vmax(Ee[x], Ha[x]);
        }
        V f = fl;
#pragma unroll
        for (int x = 0; x < K; ++x) {
          const V h = vmax(vmax(tt[x], Ee[x]), f);
          Ha[x] = h - amb2;
          f = vmax(f, Ha[x]);
        }
        fout = as_i(f);
        if (lrow == m && t == kGroup - 1) {
          const int q0 = first + 2 * kGroupsPerWave * kq, q1 = q0 + 1;
          const int off = amb - beta * (m + n);
          if (q0 < r_end) {
            const int64_t idx = a.tr ? (int64_t)c * a.ld + q0 : (int64_t)q0 * a.ld + c;
            a.scores[idx] = toi(Ha[K - 1].x) + off;
          }
          if (q1 < r_end) {
            const int64_t idx = a.tr ? (int64_t)c * a.ld + q1 : (int64_t)q1 * a.ld + c;
            a.scores[idx] = toi(Ha[K - 1].y) + off;
          }
        }
      }
      hl_prev = hl;
      selfeed = dpp_shl1(selfeed, selfeed);
    }
    selfeed = selnext;
  }
}

template <int MODE, int K, int CELL>
__global__ void __launch_bounds__(kWave) all_vs_all_i16_kernel(AllVsAllArgs a) {
  constexpr int W = kGroup * K;
  const int lane = threadIdx.x;
  const int g = lane >> 4;
  const int t = lane & 15;
  const int alpha = a.alpha, beta = a.beta;
  const int asz = a.asz;
  const int bias = (MODE == kLocal) ? alpha : alpha + beta;
  const int pad_val = (MODE == kLocal) ? alpha : (MODE == kGlobal ? alpha - beta : alpha + beta);
  const uint32_t pad_word = profile_byte<CELL>(pad_val) * 0x01010101u;
  __shared__ uint32_t ptab[8];
  if (lane < 8) {
    const int o = lane >> 2, sl = lane & 3;
    uint32_t w = 0;
    if (sl < asz)
      for (int c = 0; c < asz; ++c) {
        const int sv = o ? a.subst[sl * asz + c] : a.subst[c * asz + sl];
        w |= profile_byte<CELL>(sv + bias) << (8 * c);
      }
    ptab[lane] = w;
  }
  __syncthreads();
  const int64_t n_items = (int64_t)a.n_cols * a.n_blocks;
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(a.next, 1);
    item = __shfl(item, 0);
    if (item >= n_items) break;
    const int c = item / a.n_blocks, blk = item % a.n_blocks;
    const int64_t c0 = a.offs_c[c];
    const int n = (int)(a.offs_c[c + 1] - c0);
    const uint8_t *cols = a.seqs_c + c0;
    int bad = 0;
    // ---- the column's register profile, built once for the whole block ----
    uint32_t P[K];
#pragma unroll
    for (int x = 0; x < K; ++x) P[x] = profile_word(ptab, cols, n, a.tr != 0, t * K + x + 1 - (W - n), asz,
                                                   pad_word, bad);
    const int r_end = min(a.n_rows, (blk + 1) * a.rows_per_block);
    // (not for 512-column stripes: the extra state would push them past 256 VGPRs)
    if constexpr (MODE == kGlobal && K <= kK16) {
      if (a.eq_rows > 0 && n > 0) {
        stream_global<K, CELL>(a, P, c, n, blk * a.rows_per_block, r_end, lane, bad);
        if (bad) atomicOr(a.status, kStatusBadResidue);
        continue;
      }
    }
    for (int r = blk * a.rows_per_block; r < r_end; r += 2 * kGroupsPerWave) {
      const int q0 = r + 2 * g, q1 = q0 + 1;
      const bool has0 = q0 < r_end, has1 = q1 < r_end;
      const int64_t o0 = has0 ? a.offs_r[q0] : 0, o1 = has1 ? a.offs_r[q1] : 0;
      const int m0 = has0 ? (int)(a.offs_r[q0 + 1] - o0) : 0;
      const int m1 = has1 ? (int)(a.offs_r[q1 + 1] - o1) : 0;
      int r0, r1;
      bool over0, over1;
      duo_core<MODE, K, CELL>(a.seqs_r + o0, a.seqs_r + o1, m0, m1, n, n, P, P, asz, alpha, beta, a.sat_limit,
                              lane, bad, r0, r1, over0, over1);
      if (t == 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bool has = h ? has1 : has0;
          if (!has) continue;
          const int q = h ? q1 : q0;
          const int m = h ? m1 : m0;
          int v = h ? r1 : r0;
          const bool over = h ? over1 : over0;
          const int64_t idx = a.tr ? (int64_t)c * a.ld + q : (int64_t)q * a.ld + c;
          if (m == 0 || n == 0) {
            // an empty side: one gap run (global) or the empty alignment
            v = (MODE == kGlobal && m + n > 0) ? -alpha - beta * (m + n - 1) : 0;
          } else if (over) {
            // re-run descriptor: rows from the row sequences, columns from the
            // column sequences; "transposed" when sigma's first index is the
            // column's letter (the 32-bit launch passes the buffers to match)
            PairDesc d;
            d.row_off = a.offs_r[q];
            d.col_off = c0;
            d.m = m;
            d.n = n;
            d.pair = (int32_t)idx;
            d.flags = with_variant(a.tr ? kTransposed : 0, K > 16 ? kVarI32K32 : kVarI32K16);
            a.rerun[atomicAdd(a.n_rerun, 1)] = d;
            continue;
          }
          a.scores[idx] = v;
        }
      }
    }
    if (bad) atomicOr(a.status, kStatusBadResidue);
  }
}

template <int MODE>
hipError_t launch_mode(const FullDp16Args &args, int grid, hipStream_t stream) {
  if (args.half == kCellF16E5M2)
    hipLaunchKernelGGL((full_dp_i16_kernel<MODE, kK16, kCellF16E5M2>), dim3(grid), dim3(kWave), 0, stream, args);
  else if (args.half == kCellF16E4M3)
    hipLaunchKernelGGL((full_dp_i16_kernel<MODE, kK16, kCellF16E4M3>), dim3(grid), dim3(kWave), 0, stream, args);
  else
    hipLaunchKernelGGL((full_dp_i16_kernel<MODE, kK16, kCellI16>), dim3(grid), dim3(kWave), 0, stream, args);
  return hipGetLastError();
}

}  // namespace

int full_dp_i16_stripe_width() { return kW16; }

int full_dp_i16_blocks_per_cu(int mode) {
  int nb = 0;
  hipError_t e;
  if (mode == kGlobal)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, full_dp_i16_kernel<kGlobal, kK16, kCellI16>, kWave, 0);
  else if (mode == kSemiGlobal)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, full_dp_i16_kernel<kSemiGlobal, kK16, kCellI16>, kWave, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, full_dp_i16_kernel<kLocal, kK16, kCellI16>, kWave, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

template <int MODE, int K>
hipError_t launch_avsa_k(const AllVsAllArgs &args, int grid, hipStream_t stream) {
  if (args.half == kCellF16E5M2)
    hipLaunchKernelGGL((all_vs_all_i16_kernel<MODE, K, kCellF16E5M2>), dim3(grid), dim3(kWave), 0, stream, args);
  else if (args.half == kCellF16E4M3)
    hipLaunchKernelGGL((all_vs_all_i16_kernel<MODE, K, kCellF16E4M3>), dim3(grid), dim3(kWave), 0, stream, args);
  else
    hipLaunchKernelGGL((all_vs_all_i16_kernel<MODE, K, kCellI16>), dim3(grid), dim3(kWave), 0, stream, args);
  return hipGetLastError();
}

// Column sequences of at most 128 residues take 128-column stripes (K = 8):
// half the padding of the 256-column stripe for the paper's 125-bp reads;
// columns of 257..512 residues take 512-column stripes (K = 32).
template <int MODE>
hipError_t launch_avsa_mode(const AllVsAllArgs &args, int grid, hipStream_t stream) {
  if (args.kcols == 8) return launch_avsa_k<MODE, kK8>(args, grid, stream);
  if (args.kcols == 32) return launch_avsa_k<MODE, kK32>(args, grid, stream);
  return launch_avsa_k<MODE, kK16>(args, grid, stream);
}

hipError_t launch_all_vs_all_i16(int mode, const AllVsAllArgs &args, int grid, hipStream_t stream) {
  switch (mode) {
    case kGlobal: return launch_avsa_mode<kGlobal>(args, grid, stream);
    case kSemiGlobal: return launch_avsa_mode<kSemiGlobal>(args, grid, stream);
    default: return launch_avsa_mode<kLocal>(args, grid, stream);
  }
}

template <int K>
int avsa_occupancy(int mode) {
  int nb = 0;
  hipError_t e;
  if (mode == kGlobal)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, all_vs_all_i16_kernel<kGlobal, K, kCellI16>, kWave, 0);
  else if (mode == kSemiGlobal)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, all_vs_all_i16_kernel<kSemiGlobal, K, kCellI16>, kWave, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, all_vs_all_i16_kernel<kLocal, K, kCellI16>, kWave, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

int all_vs_all_i16_blocks_per_cu(int mode, int kcols) {
  return kcols == 8 ? avsa_occupancy<kK8>(mode) : (kcols == 32 ? avsa_occupancy<kK32>(mode) : avsa_occupancy<kK16>(mode));
}

hipError_t launch_full_dp_i16(int mode, const FullDp16Args &args, int grid, hipStream_t stream) {
  switch (mode) {
    case kGlobal: return launch_mode<kGlobal>(args, grid, stream);
    case kSemiGlobal: return launch_mode<kSemiGlobal>(args, grid, stream);
    default: return launch_mode<kLocal>(args, grid, stream);
  }
}

}  // namespace asmi
