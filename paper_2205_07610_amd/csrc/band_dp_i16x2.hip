// Banded Gotoh DP with packed 16-bit cells, global mode: two pairs per lane
// group, one in each 16-bit half of every register, so one packed VALU
// instruction updates two band cells.  Layout, recurrences and certificate
// are those of the 32-bit banded kernel (band_dp_i32.hip: sheared band of
// W = G*K diagonals, lane t owns K of them, shifted frame X + beta*(i+j),
// register 0 updated first and its (E, H') handed to lane t-1); what
// differs:
//
//  * Scores: one v_perm_b32 per cell pair.  Its sources are the two pairs'
//    row score words (byte c = sigma(row letter, c) + alpha + beta), its
//    selector [code_lo, 0, code_hi + 4, 0] picks each half's byte and
//    zero-extends it.  Each register keeps its selector word; going down a
//    row, register x takes the selector of register x+1 and the last one
//    takes lane t+1's register 1 (that lane runs one row behind) or the
//    column feed -- a rotation of the register names, free in the 16-step
//    unrolled chunks; when K does not divide 16 the chunks come in
//    K / gcd(K, 16) compile-time phases of the rotation.
//  * Columns left of column 0: in global mode no alignment path visits them,
//    so they hold -infinity (int16 saturation), and column 0 itself is then
//    produced exactly by the recurrence: E carries the corner value down,
//    which in the shifted frame is the constant boundary H'(i,0) = 2(beta -
//    alpha).  All packed arithmetic saturates, so -infinity stays put and
//    never wraps.  Columns right of n use selector 0 (score 0) and never
//    influence column n or any cell left of it.
//  * Range: a pair is queued here only when an a priori bound keeps every
//    shifted cell (band columns up to n + W) inside int16; the others take
//    the 32-bit banded kernel.
#include <type_traits>

#include "internal.h"

namespace asmi {
namespace {

typedef short s2 __attribute__((ext_vector_type(2)));

constexpr short kNeg = -32768;

__device__ __forceinline__ int as_i(s2 v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ s2 as_s2(int v) { return __builtin_bit_cast(s2, v); }
__device__ __forceinline__ s2 pk(int lo, int hi) {
  s2 r;
  r.x = (short)lo;
  r.y = (short)hi;
  return r;
}
__device__ __forceinline__ s2 vmax(s2 a, s2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s2 add_sat(s2 a, s2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ s2 sub_sat(s2 a, s2 b) { return __builtin_elementwise_sub_sat(a, b); }

template <int G>
__device__ __forceinline__ int shr1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, G == 16 ? 0x111 : 0x138, 0xF, 0xF, false);
}
template <int G>
__device__ __forceinline__ int shl1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, G == 16 ? 0x101 : 0x130, 0xF, 0xF, false);
}
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
template <int G>
__device__ __forceinline__ int wave_max_groups(int v) {
  if (G == 16) {
    v = max(v, __shfl_xor(v, 16));
    v = max(v, __shfl_xor(v, 32));
  }
  return v;
}

// Selector word of one register: byte 0 selects letter c0 of the low half's
// score word (source bytes 0..3), byte 2 letter c1 of the high half's (4..7),
// bytes 1 and 3 the constant 0; a code of 12 (no residue) selects 0.
__device__ __forceinline__ uint32_t make_sel(uint32_t c0, uint32_t c1) {
  const uint32_t s1 = c1 == 12u ? 12u : c1 + 4u;
  return c0 | 0x0C00u | (s1 << 16) | 0x0C000000u;
}

constexpr int gcd16(int k) { return k % 16 == 0 ? 16 : k % 8 == 0 ? 8 : k % 4 == 0 ? 4 : k % 2 == 0 ? 2 : 1; }

// Waves per SIMD the register allocation aims for: four for the narrowest
// class, three for the others (what the compiler would pick for the wider
// ones is two; the few values it then spills are reloaded once per pair,
// outside the DP loops).
template <int K, int G>
constexpr int kWavesPerEu = (K == 4 && G == kGroup) ? 4 : 3;

template <int K, int G>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<K, G>)))
band_dp_i16_kernel(BandArgs a, int pc) {
  constexpr int W = G * K;
  // 16-step chunks come in NR phases of the selector rotation (K / gcd(K, 16))
  constexpr int NR = K / gcd16(K);
  static_assert(NR >= 1 && NR <= 3, "rotation phases");
  constexpr int GPW = kWave / G;
  const int lane = threadIdx.x;
  const int g = lane / G;
  const int t = lane % G;
  const int alpha = a.alpha, beta = a.beta, amb = alpha - beta;
  const int asz = a.asz;
  const int cur = a.round & 1;
  const int n_list = a.ctr->n_band16[cur][pc];
  const BandItem *list = a.sorted + a.sorted_base[kBandClasses + pc];
  const s2 amb2 = pk(amb, amb);
  const s2 neg2 = pk(kNeg, kNeg);
  const int negi = as_i(neg2);
  const int kb = t * K;

  for (;;) {
    int base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr->next_band16[pc], 2 * GPW);
    base = __builtin_amdgcn_readfirstlane(base);
    if (base >= n_list) break;
    // the two pairs of this group: 0 in the low halves, 1 in the high halves
    const int item0 = base + 2 * g, item1 = item0 + 1;
    const bool has0 = item0 < n_list, has1 = item1 < n_list;
    BandItem b0{}, b1{};
    if (has0) b0 = list[item0];
    if (has1) b1 = list[item1];
    const int m0 = has0 ? b0.d.m : 0, n0 = b0.d.n, m1 = has1 ? b1.d.m : 0, n1 = b1.d.n;
    const bool tr0 = (b0.d.flags & kTransposed) != 0, tr1 = (b1.d.flags & kTransposed) != 0;
    const uint8_t *rows0 = (tr0 ? a.seqs_b : a.seqs_a) + b0.d.row_off;
    const uint8_t *cols0 = (tr0 ? a.seqs_a : a.seqs_b) + b0.d.col_off;
    const uint8_t *rows1 = (tr1 ? a.seqs_b : a.seqs_a) + b1.d.row_off;
    const uint8_t *cols1 = (tr1 ? a.seqs_a : a.seqs_b) + b1.d.col_off;
    // band limits (requested half-width, widened to W and centred)
    auto band_lo = [&](int m, int n, int w) -> int {
      const int L = min(0, n - m) - w, U = max(0, n - m) + w;
      return L - (W - (U - L + 1)) / 2;
    };
    const int lo0 = band_lo(m0, n0, b0.w), lo1 = band_lo(m1, n1, b1.w);
    const int kn0 = n0 - m0 - lo0, kn1 = n1 - m1 - lo1;  // register of column n at row m
    int bad = 0;
    auto code = [&](bool has, const uint8_t *cols, int n, int j) -> uint32_t {
      if (!has || j < 1 || j > n) return 12u;
      uint32_t c = cols[j - 1];
      if (c >= (uint32_t)asz) { bad = 1; c = 0; }
      return c;
    };
    auto qword = [&](const uint8_t *rows, int m, bool tr, int idx) -> uint32_t {
      if (idx < 0 || idx >= m) return 0u;
      int r = rows[idx];
      if (r >= asz) { bad = 1; r = 0; }
      return a.qwords[(tr ? 32 : 0) + r];
    };
    // row 0: column 0 is the corner, columns left of it are outside the matrix
    auto init1 = [&](int lo, int x) -> int {
      const int j = lo + kb + x;
      return j < 0 ? kNeg : (j == 0 ? beta - alpha : 2 * beta - 2 * alpha);
    };
    auto init_h = [&](int x) -> s2 { return pk(init1(lo0, x), init1(lo1, x)); };
    s2 Ha[K], Ee[K];
    uint32_t P[K];  // selector words; register x's is P[(x + u) % K] at step u
#pragma unroll
    for (int x = 0; x < K; ++x) {
      Ha[x] = init_h(x);
      Ee[x] = neg2;
      P[x] = make_sel(code(has0, cols0, n0, -t + lo0 + kb + x), code(has1, cols1, n1, -t + lo1 + kb + x));
    }
    int fout = negi;
    uint32_t qrow0 = 0, qrow1 = 0;
    int res0 = kNegInf32, res1 = kNegInf32;
    const int mmax = max(m0, m1);
    const int its = mmax > 0 ? mmax + G - 1 : 0;
    const int its_max = wave_max_groups<G>(its);
    uint32_t qfeed0 = qword(rows0, m0, tr0, t), qfeed1 = qword(rows1, m1, tr1, t);
    // new selectors enter at the group's last lane (element u in lane G-1-u)
    auto cfeed_at = [&](int it0) -> uint32_t {
      const int jo = it0 + (G - 1 - t) - (G - 2) + W - 1;
      return make_sel(code(has0, cols0, n0, jo + lo0), code(has1, cols1, n1, jo + lo1));
    };
    uint32_t cfeed = cfeed_at(0);
    // One chunk of 16 steps.  FILL: the pipeline is still filling (some
    // lane's row is <= 0); only the first G / 16 chunks need the test, so the
    // main loop carries none.  R0: the rotation phase (16 c mod K for chunk c).
    auto chunk = [&](int it0, auto fill_tag, auto r0_tag) __attribute__((always_inline)) {
      constexpr bool FILL = decltype(fill_tag)::value;
      constexpr int R0 = decltype(r0_tag)::value;
      const uint32_t qnext0 = qword(rows0, m0, tr0, it0 + kGroup + t);
      const uint32_t qnext1 = qword(rows1, m1, tr1, it0 + kGroup + t);
      const uint32_t cnext = cfeed_at(it0 + kGroup);
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int row = it0 + u + 1 - t;
        // this row's selectors: the register names rotate by one, and the
        // last register takes lane t+1's register 1 of the previous step --
        // lane t+1 runs one row behind, so that is this row's next column --
        // or, in the group's last lane, the column feed
        P[(u + R0) % K] = (uint32_t)shl1<G>((int)cfeed, (int)P[(u + R0 + 1) % K]);
        qrow0 = (uint32_t)shr1<G>((int)qfeed0, (int)qrow0);
        qrow1 = (uint32_t)shr1<G>((int)qfeed1, (int)qrow1);
        const s2 fl = as_s2(shr1<G>(negi, fout));
        // In the sheared layout a cell's diagonal predecessor is its own
        // register one row earlier and "up" is the next register, so the
        // update runs in place in ascending order (register x+1 is still the
        // previous row's when register x reads it).  Register 0 goes first and
        // its (E, H') moves to lane t-1 before the others.
        // While the pipeline fills, a lane whose row is still <= 0 skips the
        // update (a branch on the execution mask), so its registers keep the
        // row-0 values set before the loop and its outputs to the neighbour
        // lanes are row 0's.
        const bool live = !FILL || row > 0;
        s2 f = fl;
        if (live) {
          const s2 sc = as_s2((int)__builtin_amdgcn_perm(qrow1, qrow0, P[(u + R0 + 1) % K]));
          const s2 e = K > 1 ? vmax(Ee[1], Ha[1]) : neg2;
          const s2 hv = vmax(vmax(add_sat(Ha[0], sc), e), f);
          Ha[0] = sub_sat(hv, amb2);
          Ee[0] = e;
          f = vmax(f, Ha[0]);
        }
        const s2 eR = as_s2(shl1<G>(negi, as_i(vmax(Ee[0], Ha[0]))));
        if (live) {
#pragma unroll
          for (int x = 1; x < K; ++x) {
            const s2 sc = as_s2((int)__builtin_amdgcn_perm(qrow1, qrow0, P[(x + u + R0 + 1) % K]));
            const s2 e = (x + 1 < K) ? vmax(Ee[x + 1], Ha[x + 1]) : eR;
            const s2 hv = vmax(vmax(add_sat(Ha[x], sc), e), f);
            Ha[x] = sub_sat(hv, amb2);
            Ee[x] = e;
            f = vmax(f, Ha[x]);
          }
        }
        fout = live ? as_i(f) : negi;
        // a pair's last row: H(m, n) sits in register kn of lane kn / K
        if (__builtin_amdgcn_ballot_w64(row == m0 || row == m1) != 0) {
          if (row == m0 && kn0 / K == t) {
#pragma unroll
            for (int x = 0; x < K; ++x)
              if (x == kn0 % K) res0 = (int)Ha[x].x + amb - beta * (m0 + n0);
          }
          if (row == m1 && kn1 / K == t) {
#pragma unroll
            for (int x = 0; x < K; ++x)
              if (x == kn1 % K) res1 = (int)Ha[x].y + amb - beta * (m1 + n1);
          }
        }
        qfeed0 = (uint32_t)shl1<G>((int)qfeed0, (int)qfeed0);
        qfeed1 = (uint32_t)shl1<G>((int)qfeed1, (int)qfeed1);
        cfeed = (uint32_t)shr1<G>((int)cfeed, (int)cfeed);
      }
      qfeed0 = qnext0;
      qfeed1 = qnext1;
      cfeed = cnext;
    };
    auto phase = [&](int it0, int c, auto fill_tag) __attribute__((always_inline)) {
      const int ph = NR == 1 ? 0 : c % NR;
      if (ph == 0) chunk(it0, fill_tag, std::integral_constant<int, 0>{});
      else if (NR > 1 && ph == 1) chunk(it0, fill_tag, std::integral_constant<int, kGroup % K>{});
      else if (NR > 2) chunk(it0, fill_tag, std::integral_constant<int, (2 * kGroup) % K>{});
    };
    int it0 = 0, c = 0;
    for (; it0 < its_max && it0 < G; it0 += kGroup, ++c) phase(it0, c, std::true_type{});
    for (; it0 < its_max; it0 += kGroup, ++c) phase(it0, c, std::false_type{});

    const int score0 = group_max<G>(res0), score1 = group_max<G>(res1);
    if (bad) atomicOr(&a.ctr->status, kStatusBadResidue);
    // lane 0 settles the low half's pair, lane 1 the high half's
    if (t > 1) continue;
    const bool has = t == 0 ? has0 : has1;
    if (!has) continue;
    PairDesc d;  // field by field: a whole-struct select would go through scratch memory
    d.row_off = t == 0 ? b0.d.row_off : b1.d.row_off;
    d.col_off = t == 0 ? b0.d.col_off : b1.d.col_off;
    d.m = t == 0 ? b0.d.m : b1.d.m;
    d.n = t == 0 ? b0.d.n : b1.d.n;
    d.pair = t == 0 ? b0.d.pair : b1.d.pair;
    d.flags = t == 0 ? b0.d.flags : b1.d.flags;
    const int w = t == 0 ? b0.w : b1.w;
    const int score = t == 0 ? score0 : score1;
    const int m = d.m, n = d.n, lo = t == 0 ? lo0 : lo1, hi = lo + W - 1;
    int64_t ub = 0;
    const bool leave = band_leave_bound(m, n, lo, hi, a.sigma_max, alpha, beta, kGlobal, &ub);
    atomicAdd(&a.ctr->band_cells, (unsigned long long)((long long)m * W));
    atomicAdd(&a.ctr->band16_cells, (unsigned long long)((long long)m * W));
    if (!leave || (int64_t)score >= ub) {
      a.scores[d.pair] = score;
      atomicAdd(&a.ctr->band_accepted[a.round < kMaxBandRounds ? a.round : kMaxBandRounds - 1], 1);
      continue;
    }
    band_requeue(a, d, w, kGlobal, W);
  }
}

template <int K, int G>
int occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, band_dp_i16_kernel<K, G>, kWave, 0) != hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

}  // namespace

// Packed classes (widths 1.5x or 1.33x apart): 64, 96, 128, 192, 256
// diagonals on 16-lane groups (K = 4, 6, 8, 12, 16; eight pairs per wave),
// 384, 512, 768, 1024 on whole waves (K = 6, 8, 12, 16; two pairs).
#define AS_BAND16_CLASSES(X) \
  X(0, 4, 16) X(1, 6, 16) X(2, 8, 16) X(3, 12, 16) X(4, 16, 16) X(5, 6, 64) X(6, 8, 64) X(7, 12, 64) X(8, 16, 64)

hipError_t launch_band_dp_i16(int pc, const BandArgs &args, int grid, hipStream_t stream) {
  switch (pc) {
#define AS_LAUNCH(PC, K, G) \
  case PC: hipLaunchKernelGGL((band_dp_i16_kernel<K, G>), dim3(grid), dim3(kWave), 0, stream, args, pc); break;
    AS_BAND16_CLASSES(AS_LAUNCH)
#undef AS_LAUNCH
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int band_dp_i16_blocks_per_cu(int pc) {
  switch (pc) {
#define AS_OCC(PC, K, G) \
  case PC: return occupancy<K, G>();
    AS_BAND16_CLASSES(AS_OCC)
#undef AS_OCC
    default: return 1;
  }
}

int band_dp_i16_pairs_per_wave(int pc) { return band16_class_lanes(pc) == kWave ? 2 : 2 * kGroupsPerWave; }

}  // namespace asmi
