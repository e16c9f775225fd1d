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
//    takes lane t+1's register 1 (that lane runs one row behind) or, in the
//    group's last lane, the selector of the column entering the band -- a
//    rotation of the register names, free in the unrolled chunks of CH
//    steps (32, or 24 / 48 when K is 6 or 12: CH is a multiple of K).
//  * Feeds through LDS: at the start of each chunk the group's lanes write
//    the score words of the chunk's CH new rows into a ring of rows (its
//    first CH slots mirrored past its end, so a lane's CH reads of a chunk
//    are contiguous and take the step from the instruction's offset) and
//    the selectors of the CH entering columns; the residues were loaded one
//    chunk ahead.  A step then costs the cell updates, two LDS reads and
//    three DPP moves.
//  * Values are stored with a bias as unsigned 16-bit numbers, so 0 is
//    -infinity (the bias is 32768, or lower for a pair whose upper bound
//    needs the room: band16_bias): DPP moves that shift in from outside the group write 0
//    themselves, and all packed arithmetic saturates, so -infinity stays put
//    and never wraps.  Columns left of column 0 hold -infinity (in global
//    mode no alignment path visits them) and column 0 itself is produced
//    exactly by the recurrence: E carries the corner value down, which in
//    the shifted frame is the constant boundary H'(i,0) = 2(beta - alpha).
//    Columns right of n use selector 0 (score 0) and never influence column
//    n or any cell left of it.
//  * Results: a chunk in which some lane reaches a pair's last row runs a
//    variant with the per-step test for H(m, n); the others carry none.
//  * Range: a pair is queued here only when an a priori bound keeps every
//    shifted cell (band columns up to n + W) inside int16; the others take
//    the 32-bit banded kernel.
//  * Raw mode writes each pair's banded score and the band's limits and
//    queues nothing.
#include <type_traits>

#include "internal.h"

namespace asmi {
namespace {

typedef unsigned short u2 __attribute__((ext_vector_type(2)));


__device__ __forceinline__ int as_i(u2 v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ u2 as_u2(int v) { return __builtin_bit_cast(u2, v); }
__device__ __forceinline__ u2 pk(int lo, int hi) {
  u2 r;
  r.x = (unsigned short)lo;
  r.y = (unsigned short)hi;
  return r;
}
__device__ __forceinline__ u2 vmax(u2 a, u2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ u2 add_sat(u2 a, u2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ u2 sub_sat(u2 a, u2 b) { return __builtin_elementwise_sub_sat(a, b); }

// Group-local shifts by one lane: shr1z/shl1z write 0 where the source lane
// is outside the group; shl1 keeps `old` there.
template <int G>
__device__ __forceinline__ int shr1z(int src) {
  return __builtin_amdgcn_update_dpp(0, src, G == 16 ? 0x111 : 0x138, 0xF, 0xF, true);
}
template <int G>
__device__ __forceinline__ int shl1z(int src) {
  return __builtin_amdgcn_update_dpp(0, src, G == 16 ? 0x101 : 0x130, 0xF, 0xF, true);
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

// Steps per unrolled chunk: a multiple of K, so the selector rotation
// returns to the identity at every chunk boundary: 32 when K divides it,
// else about 24-30 on 16-lane groups (whose registers are already scarce)
// and 40-48 on whole waves.
constexpr int chunk_steps(int K, int G) {
  return 32 % K == 0 ? 32
       : G == kGroup ? (K == 5 ? 25 : K == 7 || K == 14 ? 28 : K == 10 ? 30 : 24)
                     : (K == 7 || K == 14 ? 42 : K == 5 || K == 10 || K == 20 ? 40 : 48);
}

// Waves per SIMD the register allocation aims for: two for K = 20 and 24
// (their state alone fills three waves' registers) and for K = 10..14 on
// 16-lane groups (K = 12 measured 8% faster than three with spills); three
// for the others (what the compiler would pick for the wider ones is two;
// the few values it then spills are reloaded once per pair, outside the DP
// loops, and two waves measured slower for K = 16).
template <int K, int G>
constexpr int kWavesPerEu = (K >= 20 || (K >= 10 && K <= 14 && G == kGroup)) ? 2 : 3;

template <int K, int G>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<K, G>)))
band_dp_i16_kernel(BandArgs a, int pc) {
  constexpr int W = G * K;
  constexpr int CH = chunk_steps(K, G);
  static_assert(CH % K == 0, "the rotation must close over a chunk");
  // rows a chunk reads span G + CH - 1; the next chunk's CH are written past them
  constexpr int kRing = (G + 2 * CH <= 128) ? 128 : 256;
  constexpr int NF = (CH + G - 1) / G;  // rows (and entering columns) each lane feeds per chunk
  constexpr int GPW = kWave / G;
  __shared__ uint2 rq[GPW][kRing + CH];  // row words (low pair, high pair) by row mod kRing
  __shared__ uint32_t sq[GPW][CH];       // selectors entering at the last lane, by step of the chunk
  __shared__ uint32_t qt[8];                 // score word by (orientation, letter)
  const int lane = threadIdx.x;
  const int g = lane / G;
  const int t = lane % G;
  const int alpha = a.alpha, beta = a.beta, amb = alpha - beta;
  const uint32_t asz = (uint32_t)a.asz;  // at most 4 on this path
  const int cur = a.round & 1;
  const int n_list = a.ctr->n_band16[cur][pc];
  const BandItem *list = a.sorted + a.sorted_base[kBandClasses + pc];
  const u2 amb2 = pk(amb, amb);
  const int kb = t * K;
  if (lane < 8) qt[lane] = a.qwords[(lane >> 2) * 32 + (lane & 3)];
  __builtin_amdgcn_wave_barrier();

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
    // the step at which this lane holds H(m, n) of each half (-1: never)
    const int e0 = (has0 && t == kn0 / K) ? m0 - 1 + t : -1;
    const int e1 = (has1 && t == kn1 / K) ? m1 - 1 + t : -1;
    int bad = 0;
    // loads are clamped into the sequence so that they can be issued early;
    // what they mean is decided where they are used
    auto col_byte = [&](const uint8_t *cols, int n, int j) -> uint32_t {
      return cols[min(max(j - 1, 0), max(n - 1, 0))];
    };
    auto col_code = [&](bool has, int n, int j, uint32_t c) -> uint32_t {
      if (!has || j < 1 || j > n) return 12u;
      if (c >= asz) { bad = 1; c = 0; }
      return c;
    };
    auto row_byte = [&](const uint8_t *rows, int m, int idx) -> uint32_t {
      return rows[min(max(idx, 0), max(m - 1, 0))];
    };
    auto row_word = [&](int m, bool tr, int idx, uint32_t r) -> uint32_t {
      if (idx < 0 || idx >= m) return 0u;
      if (r >= asz) { bad = 1; r = 0; }
      return qt[(tr ? 4 : 0) + r];
    };
    // row 0: column 0 is the corner, columns left of it are outside the matrix
    const int bias0 = band16_bias(m0, n0, W, a.smax_pos, alpha, beta);
    const int bias1 = band16_bias(m1, n1, W, a.smax_pos, alpha, beta);
    auto init1 = [&](int lo, int bias, int x) -> int {
      const int j = lo + kb + x;
      return j < 0 ? 0 : bias + (j == 0 ? beta - alpha : 2 * beta - 2 * alpha);
    };
    u2 Ha[K], Ee[K];
    uint32_t P[K];  // selector words; register x's is P[(x + u) % K] at step u
#pragma unroll
    for (int x = 0; x < K; ++x) {
      Ha[x] = pk(init1(lo0, bias0, x), init1(lo1, bias1, x));
      Ee[x] = pk(0, 0);
      const int j0 = -t + lo0 + kb + x, j1 = -t + lo1 + kb + x;
      P[x] = make_sel(col_code(has0, n0, j0, col_byte(cols0, n0, j0)),
                      col_code(has1, n1, j1, col_byte(cols1, n1, j1)));
    }
    int fout = 0;
    int res0 = kNegInf32, res1 = kNegInf32;
    const int mmax = max(m0, m1);
    const int its = mmax > 0 ? mmax + G - 1 : 0;
    const int its_max = wave_max_groups<G>(its);
    // column entering the band at the group's last lane at step it
    constexpr int kEnter = W - G + 1;
    // residues of the chunk starting at it0, loaded one chunk ahead: lane t
    // feeds steps s = t + G f (f < NF, s < CH), i.e. row it0 + 1 + s and the
    // column entering at step it0 + s
    uint32_t rb0[NF], rb1[NF], cb0[NF], cb1[NF];
    auto prefetch = [&](int it0) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int s = t + G * f;
        if (s < CH) {
          rb0[f] = row_byte(rows0, m0, it0 + s);
          rb1[f] = row_byte(rows1, m1, it0 + s);
          cb0[f] = col_byte(cols0, n0, it0 + s + lo0 + kEnter);
          cb1[f] = col_byte(cols1, n1, it0 + s + lo1 + kEnter);
        }
      }
    };
    auto feed = [&](int it0) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int s = t + G * f;
        if (s < CH) {
          const int r = it0 + 1 + s;
          uint2 v;
          v.x = row_word(m0, tr0, r - 1, rb0[f]);
          v.y = row_word(m1, tr1, r - 1, rb1[f]);
          const int slot = r & (kRing - 1);
          rq[g][slot] = v;
          if (slot < CH) rq[g][slot + kRing] = v;
          const int j0 = it0 + s + lo0 + kEnter, j1 = it0 + s + lo1 + kEnter;
          sq[g][s] = make_sel(col_code(has0, n0, j0, cb0[f]), col_code(has1, n1, j1, cb1[f]));
        }
      }
      __builtin_amdgcn_wave_barrier();
    };
    prefetch(0);
    // One chunk of CH steps.  FILL: the pipeline is still filling (some
    // lane's row is <= 0); only the chunks starting before step G need the
    // test.  EXT: some lane reaches a pair's last row in this chunk.
    auto chunk = [&](int it0, auto fill_tag, auto ext_tag) __attribute__((always_inline)) {
      constexpr bool FILL = decltype(fill_tag)::value;
      constexpr bool EXT = decltype(ext_tag)::value;
      constexpr int R0 = 0;
      feed(it0);
      prefetch(it0 + CH);
      const uint2 *rrow = &rq[g][(it0 + 1 - t) & (kRing - 1)];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int row = it0 + u + 1 - t;
        // this row's selectors: the register names rotate by one, and the
        // last register takes lane t+1's register 1 of the previous step --
        // lane t+1 runs one row behind, so that is this row's next column --
        // or, in the group's last lane, the entering column's
        P[(u + R0) % K] = (uint32_t)shl1<G>((int)sq[g][u], (int)P[(u + R0 + 1) % K]);
        const uint2 q = rrow[u];
        const u2 fl = as_u2(shr1z<G>(fout));
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
        u2 f = fl;
        if (live) {
          const u2 sc = as_u2((int)__builtin_amdgcn_perm(q.y, q.x, P[(u + R0 + 1) % K]));
          const u2 e = K > 1 ? vmax(Ee[1], Ha[1]) : pk(0, 0);
          const u2 hv = vmax(vmax(add_sat(Ha[0], sc), e), f);
          Ha[0] = sub_sat(hv, amb2);
          Ee[0] = e;
          f = vmax(f, Ha[0]);
        }
        const u2 eR = as_u2(shl1z<G>(as_i(vmax(Ee[0], Ha[0]))));
        if (live) {
#pragma unroll
          for (int x = 1; x < K; ++x) {
            const u2 sc = as_u2((int)__builtin_amdgcn_perm(q.y, q.x, P[(x + u + R0 + 1) % K]));
            const u2 e = (x + 1 < K) ? vmax(Ee[x + 1], Ha[x + 1]) : eR;
            const u2 hv = vmax(vmax(add_sat(Ha[x], sc), e), f);
            Ha[x] = sub_sat(hv, amb2);
            Ee[x] = e;
            f = vmax(f, Ha[x]);
          }
        }
        fout = live ? as_i(f) : 0;
        if (EXT) {  // a pair's last row: H(m, n) sits in register kn of lane kn / K
          if (it0 + u == e0) {
#pragma unroll
            for (int x = 0; x < K; ++x)
              if (x == kn0 % K) res0 = (int)Ha[x].x - bias0 + amb - beta * (m0 + n0);
          }
          if (it0 + u == e1) {
#pragma unroll
            for (int x = 0; x < K; ++x)
              if (x == kn1 % K) res1 = (int)Ha[x].y - bias1 + amb - beta * (m1 + n1);
          }
        }
      }
      __builtin_amdgcn_wave_barrier();  // this chunk's LDS reads stay before the next feed
    };
    auto ends_in = [&](int it0) -> bool {
      return __builtin_amdgcn_ballot_w64((e0 >= it0 && e0 < it0 + CH) || (e1 >= it0 && e1 < it0 + CH)) != 0;
    };
    int it0 = 0;
    for (; it0 < its_max && it0 < G; it0 += CH) chunk(it0, std::true_type{}, std::true_type{});
    for (; it0 < its_max; it0 += CH) {
      if (__builtin_expect(ends_in(it0), 0)) chunk(it0, std::false_type{}, std::true_type{});
      else chunk(it0, std::false_type{}, std::false_type{});
    }

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
    if (a.raw) {  // the band's score and limits (A/B orientation), no rounds
      const bool tr = (d.flags & kTransposed) != 0;
      a.scores[d.pair] = score;
      if (a.lo_out) {
        a.lo_out[d.pair] = tr ? -hi : lo;
        a.hi_out[d.pair] = tr ? -lo : hi;
      }
      if (a.accept_out) a.accept_out[d.pair] = (!leave || (int64_t)score >= ub) ? 1 : 0;
      continue;
    }
    atomicAdd(&a.ctr->band_cells, (unsigned long long)((long long)m * W));
    atomicAdd(&a.ctr->band16_cells, (unsigned long long)((long long)m * W));
    if (!leave || (int64_t)score >= ub) {
      a.scores[d.pair] = score;
      atomicAdd(&a.ctr->band_accepted[a.round < kMaxBandRounds ? a.round : kMaxBandRounds - 1], 1);
      continue;
    }
    band_requeue(a, d, w, kGlobal, W, score);
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

// Packed classes (band16_class_k): 80..256 diagonals on 16-lane groups
// (K = 5, 6, 7, 8, 10, 12, 14, 16; eight pairs per wave), 320..1536 on
// whole waves (K = 5, 6, 7, 8, 10, 12, 14, 16, 20, 24; two pairs).
#define AS_BAND16_CLASSES(X)                                                                             \
  X(0, 5, 16) X(1, 6, 16) X(2, 7, 16) X(3, 8, 16) X(4, 10, 16) X(5, 12, 16) X(6, 14, 16) X(7, 16, 16)     \
      X(8, 5, 64) X(9, 6, 64) X(10, 7, 64) X(11, 8, 64) X(12, 10, 64) X(13, 12, 64) X(14, 14, 64)         \
          X(15, 16, 64) X(16, 20, 64) X(17, 24, 64)

#define AS_CHECK(PC, K, G) \
  static_assert(band16_class_k(PC) == K && band16_class_lanes(PC) == G, "packed class table");
AS_BAND16_CLASSES(AS_CHECK)
#undef AS_CHECK
static_assert(kBand16Classes == 18, "packed class list");

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
