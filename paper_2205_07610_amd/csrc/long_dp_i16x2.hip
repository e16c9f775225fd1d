// Long pairs, global mode, packed 16-bit cells: the anti-diagonal wavefront
// of long_dp_i32.hip with two pairs per wave, one in each 16-bit half of
// every register, so one packed VALU instruction updates two cells.
//
// A duo is two consecutive items of the list (ordered by stripe and row
// count, so they have about the same shape); it runs S = ceil(max(n0, n1) /
// 1024) stripes of W = 64 K columns (64 lanes x K registers, K the smallest
// count in 10..16 whose S stripes cover max(n0, n1); the routing sends only
// pairs of more than 1024 columns, so S >= 2) over max(m0, m1) rows,
// and each stripe is one task of the persistent ticket queue.  What is
// shared with the 32-bit wavefront: lane t owns K adjacent columns and in step `it`
// computes row it + 1 - t; H' and F of lane t-1 arrive through DPP
// wave_shr:1; stripe s + 1 consumes the boundary column (H', F per row)
// that stripe s publishes through memory with device-coherent accesses and
// a row counter, waiting with a bounded spin; tickets are taken in order, so
// a stripe only waits for one that an earlier ticket started.  What is new:
//
//  * Scores: the column selectors are fixed per register for a stripe
//    (make_sel of the two halves' column letters); the row's score words
//    (byte c = sigma(row letter, c) + alpha + beta) come from LDS, so one
//    v_perm_b32 gives both halves' scores.
//  * Feeds through LDS: at the start of each 32-step chunk, lanes 0..31
//    write the chunk's rows into a ring of 128 rows: the two row words and
//    the left boundary (H', F) of both halves, imported from the previous
//    stripe or, in stripe 0, the constant global boundary.  Its first 32
//    slots are mirrored past its end, so a lane's reads of a chunk are
//    contiguous; lane 0's read of row r carries both its row words and the
//    boundary it shifts in.  Residues and boundary rows are loaded one chunk
//    ahead.
//  * Export: lane 63's (H', F) of each row are staged in LDS during a chunk
//    and leave at its end as one contiguous 256-byte block (32 lanes, 8
//    bytes each), so the device-coherent stores write whole cache lines
//    instead of one partial line per row.
//  * Values carry a bias of 32768 as unsigned 16-bit numbers (0 is
//    -infinity) with saturating arithmetic; a duo is queued here only when
//    an a priori bound keeps every shifted cell inside int16.  Columns past
//    a half's n select score 0 and rows past its m select the zero row word:
//    both only lower cells and never reach column n or row m.
//  * Results: H(m, n) of each half sits in its last stripe, in lane
//    ((n - 1) mod W) / K, register (n - 1) mod K, at step m - 1 + lane; only
//    chunks that contain such a step carry the test.
#include <type_traits>

#include "internal.h"

namespace asmi {
namespace {

typedef unsigned short u2 __attribute__((ext_vector_type(2)));

constexpr int kW = kLong16Width;  // most columns per stripe (64 lanes x 16 registers)
constexpr int kCh = 32;            // steps per chunk
constexpr int kRing = 128;         // rows in the ring
constexpr int kBias = 32768;
constexpr unsigned kSpinLimit = 1u << 25;
static_assert(kRing >= kWave + 2 * kCh, "the ring holds a chunk's rows and the next chunk's");

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
// wave_shr:1 -- lane t reads lane t-1; lane 0 keeps `old`
__device__ __forceinline__ int wave_shr1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int wave_max(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ uint32_t make_sel(uint32_t c0, uint32_t c1) {
  const uint32_t s1 = c1 == 12u ? 12u : c1 + 4u;
  return c0 | 0x0C00u | (s1 << 16) | 0x0C000000u;
}
__device__ __forceinline__ void store_bnd(uint2 *p, uint32_t h, uint32_t f) {
  const unsigned long long v = (unsigned long long)h | ((unsigned long long)f << 32);
  __hip_atomic_store((unsigned long long *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint2 load_bnd(const uint2 *p) {
  const unsigned long long v =
      __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}
__device__ __forceinline__ int wait_rows(int *flag, int need, int *status) {
  int seen = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned spins = 0;
  while (seen < need) {
    __builtin_amdgcn_s_sleep(2);
    seen = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (++spins > kSpinLimit) {
      atomicOr(status, kStatusStall);
      return need;  // give up waiting; the call reports an error
    }
  }
  __asm__ __volatile__("" ::: "memory");
  return seen;
}
__device__ __forceinline__ void publish_rows(int *flag, int rows) {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_store(flag, rows, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// What one stripe task needs besides its K: the duo, the stripe and the
// block-wide constants.
struct Task {
  PairDesc d0, d1;
  bool has1;
  int s, S;        // stripe index and the duo's stripe count
  int task0;       // ticket of the duo's first stripe
  int64_t bnd_off; // the duo's first boundary entry
};

// One stripe of W = 64 K columns.  The duo's stripe count S is fixed by the
// 1024-column maximum; K is the smallest register count whose S stripes
// cover the longer half, so the padding past n is under 64 columns per
// stripe instead of up to a whole stripe.
template <int K>
__device__ __forceinline__ void stripe_task(const Long16Args &a, const Task &T, uint4 *rq, uint2 *xq,
                                            const uint32_t *qt, int t, int gb) {
  constexpr int W = kWave * K;
  const int alpha = a.alpha, beta = a.beta, amb = alpha - beta;
  const uint32_t asz = (uint32_t)a.asz;
  const u2 amb2 = pk(amb, amb);
  const uint32_t gb2 = (uint32_t)as_i(pk(gb, gb));
  const PairDesc &d0 = T.d0, &d1 = T.d1;
  const bool has1 = T.has1;
  const int s = T.s, S = T.S;
  const int m0 = d0.m, n0 = d0.n, m1 = has1 ? d1.m : 0, n1 = has1 ? d1.n : 0;
  const int mmax = max(m0, m1);
  const bool tr0 = (d0.flags & kTransposed) != 0, tr1 = (d1.flags & kTransposed) != 0;
  const uint8_t *rows0 = (tr0 ? a.seqs_b : a.seqs_a) + d0.row_off;
  const uint8_t *cols0 = (tr0 ? a.seqs_a : a.seqs_b) + d0.col_off;
  const uint8_t *rows1 = (tr1 ? a.seqs_b : a.seqs_a) + d1.row_off;
  const uint8_t *cols1 = (tr1 ? a.seqs_a : a.seqs_b) + d1.col_off;
  const bool import = s > 0;
  const bool export_ = s + 1 < S;
  const uint2 *bin = a.bnd + T.bnd_off + (int64_t)(s - 1) * (mmax + 1);
  uint2 *bout = a.bnd + T.bnd_off + (int64_t)s * (mmax + 1);
  int *flag_in = a.flags + T.task0 + s - 1;
  int *flag_out = a.flags + T.task0 + s;
  int bad = 0;

  // ---- column selectors of this lane's K columns ----
  const int jp0 = s * W + t * K;  // columns jp0 + 1 .. jp0 + K
  auto col_code = [&](const uint8_t *cols, int n, int j) -> uint32_t {
    if (j < 1 || j > n) return 12u;
    uint32_t c = cols[j - 1];
    if (c >= asz) { bad = 1; c = 0; }
    return c;
  };
  uint32_t P[K];
#pragma unroll
  for (int x = 0; x < K; ++x)
    P[x] = make_sel(col_code(cols0, n0, jp0 + x + 1), has1 ? col_code(cols1, n1, jp0 + x + 1) : 12u);
  // ---- row-0 state (shifted frame, global): H'(0, j) = 2 (beta - alpha) for j >= 1 ----
  u2 Ha[K], Ee[K];
#pragma unroll
  for (int x = 0; x < K; ++x) {
    Ha[x] = pk(gb, gb);
    Ee[x] = pk(0, 0);
  }
  // diagonal of (1, jp0 + 1): H'(0, jp0), the corner H'(0, 0) = beta - alpha
  const int c0v = jp0 == 0 ? kBias + beta - alpha : gb;
  u2 hl_prev = pk(c0v, c0v);
  int hout = as_i(Ha[K - 1]);
  int fout = 0;
  // results: step at which this lane holds H(m, n) of each half (-1: never)
  const int S0 = (n0 + W - 1) / W, S1 = (n1 + W - 1) / W;
  const int tc0 = ((n0 - 1) % W) / K, xc0 = (n0 - 1) % K;
  const int tc1 = ((n1 - 1) % W) / K, xc1 = (n1 - 1) % K;
  const int e0 = (s == S0 - 1 && t == tc0) ? m0 - 1 + t : -1;
  const int e1 = (has1 && s == S1 - 1 && t == tc1) ? m1 - 1 + t : -1;
  int res0 = kNegInf32, res1 = kNegInf32;

  // ---- feeds: lane t < kCh feeds row it0 + 1 + t, loaded one chunk ahead ----
  uint32_t rb0 = 0, rb1 = 0;
  uint2 bb = make_uint2(0, 0);
  int seen = 0;  // rows the producer is known to have published
  auto prefetch = [&](int it0) {
    if (import && it0 + 1 <= mmax) {
      const int need = min(it0 + kCh, mmax);
      if (seen < need) seen = wait_rows(flag_in, need, &a.ctr->status);
    }
    if (t < kCh) {
      const int r = it0 + 1 + t;  // row, 1-based
      rb0 = rows0[min(max(r - 1, 0), max(m0 - 1, 0))];
      rb1 = has1 ? rows1[min(max(r - 1, 0), max(m1 - 1, 0))] : 0u;
      if (import && r <= mmax) bb = load_bnd(bin + r);
    }
  };
  auto feed = [&](int it0) {
    if (t < kCh) {
      const int r = it0 + 1 + t;
      uint4 v;
      uint32_t c0 = rb0, c1 = rb1;
      if (r <= m0 && c0 >= asz) { bad = 1; c0 = 0; }
      if (r <= m1 && c1 >= asz) { bad = 1; c1 = 0; }
      v.x = r <= m0 ? qt[(tr0 ? 4 : 0) + c0] : 0u;
      v.y = r <= m1 ? qt[(tr1 ? 4 : 0) + c1] : 0u;
      v.z = import ? bb.x : gb2;
      v.w = import ? bb.y : gb2;
      const int slot = r & (kRing - 1);
      rq[slot] = v;
      if (slot < kCh) rq[slot + kRing] = v;
    }
    __builtin_amdgcn_wave_barrier();
  };
  const int its = mmax + kWave - 1;
  prefetch(0);
  auto chunk = [&](int it0, auto fill_tag, auto ext_tag) __attribute__((always_inline)) {
    constexpr bool FILL = decltype(fill_tag)::value;
    constexpr bool EXT = decltype(ext_tag)::value;
    feed(it0);
    prefetch(it0 + kCh);
    const uint4 *rrow = &rq[(it0 + 1 - t) & (kRing - 1)];
#pragma unroll
    for (int u = 0; u < kCh; ++u) {
      const int row = it0 + u + 1 - t;
      const uint4 q = rrow[u];
      // H' and F of the column left of this lane's first: lane t-1's last
      // of this row, or, in lane 0, the boundary of the row
      const u2 hl = as_u2(wave_shr1((int)q.z, hout));
      const u2 fl = as_u2(wave_shr1((int)q.w, fout));
      const bool live = !FILL || row > 0;
      if (live) {
        // phase A, independent per column: diagonal sums from the previous
        // row, E from the previous row's H'
        u2 tt[K];
#pragma unroll
        for (int x = 0; x < K; ++x) {
          const u2 sc = as_u2((int)__builtin_amdgcn_perm(q.y, q.x, P[x]));
          tt[x] = add_sat(x == 0 ? hl_prev : Ha[x - 1], sc);
          Ee[x] = vmax(Ee[x], Ha[x]);
        }
        // phase B, the F chain along the row
        u2 f = fl;
#pragma unroll
        for (int x = 0; x < K; ++x) {
          const u2 h = vmax(vmax(tt[x], Ee[x]), f);
          Ha[x] = sub_sat(h, amb2);
          f = vmax(f, Ha[x]);
        }
        hout = as_i(Ha[K - 1]);
        fout = as_i(f);
        if (export_ && t == kWave - 1) xq[u] = make_uint2((uint32_t)hout, (uint32_t)fout);
      }
      hl_prev = hl;
      if (EXT) {
        if (it0 + u == e0) {
#pragma unroll
          for (int x = 0; x < K; ++x)
            if (x == xc0) res0 = (int)Ha[x].x - kBias + amb - beta * (m0 + n0);
        }
        if (it0 + u == e1) {
#pragma unroll
          for (int x = 0; x < K; ++x)
            if (x == xc1) res1 = (int)Ha[x].y - kBias + amb - beta * (m1 + n1);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();  // this chunk's LDS reads stay before the next feed
    if (export_) {
      // the chunk's exported rows leave as one contiguous block (lane u
      // stores the row lane 63 finished at step it0 + u); then every
      // complete row is published
      if (t < kCh) {
        const int row = it0 + t - (kWave - 2);
        if (row >= 1 && row <= mmax) {
          const uint2 v = xq[t];
          store_bnd(bout + row, v.x, v.y);
        }
      }
      const int done = min(it0 + kCh - (kWave - 1), mmax);
      if (done > 0) publish_rows(flag_out, done);
    }
  };
  auto ends_in = [&](int it0) -> bool {
    return __builtin_amdgcn_ballot_w64((e0 >= it0 && e0 < it0 + kCh) || (e1 >= it0 && e1 < it0 + kCh)) != 0;
  };
  int it0 = 0;
  for (; it0 < its && it0 < kWave; it0 += kCh) chunk(it0, std::true_type{}, std::true_type{});
  for (; it0 < its; it0 += kCh) {
    if (__builtin_expect(ends_in(it0), 0)) chunk(it0, std::false_type{}, std::true_type{});
    else chunk(it0, std::false_type{}, std::false_type{});
  }
  if (export_) publish_rows(flag_out, mmax);

  const int r0 = wave_max(res0), r1 = wave_max(res1);
  if (t == 0) {
    if (s == S0 - 1) a.scores[d0.pair] = r0;
    if (has1 && s == S1 - 1) a.scores[d1.pair] = r1;
  }
  if (bad) atomicOr(&a.ctr->status, kStatusBadResidue);
}

// Registers per lane for a duo whose longer half has n columns in S stripes
// (at least 10: pairs here have more than 1024 columns, hence K >= 9).
__host__ __device__ inline int stripe_k(int n, int S) {
  const int k = (n + kWave * S - 1) / (kWave * S);
  return k <= 10 ? 10 : k;
}

__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3)))
long_dp_i16_kernel(Long16Args a) {
  __shared__ uint4 rq[kRing + kCh];  // per row: row words (low, high pair), boundary H', F
  __shared__ uint2 xq[kCh];          // the exported column of one chunk: H', F of both halves
  __shared__ uint32_t qt[8];         // score word by (orientation, letter)
  const int t = threadIdx.x;
  const int alpha = a.alpha, beta = a.beta;
  const int n_tasks = a.ctr->n_long16_tasks;
  const int n_items = a.ctr->n_long16;
  const int n_duos = (n_items + 1) / 2;
  if (t < 8) {  // word of row letter r: byte c = sigma(r, c) + alpha + beta (orientation t >> 2)
    const int o = t >> 2, r = t & 3;
    uint32_t w = 0;
    if (r < a.asz)
      for (int c = 0; c < a.asz; ++c) {
        const int sv = o == 0 ? a.subst[r * a.asz + c] : a.subst[c * a.asz + r];
        w |= (uint32_t)((sv + alpha + beta) & 0xFF) << (8 * c);
      }
    qt[t] = w;
  }
  __builtin_amdgcn_wave_barrier();
  // the global boundary column in the shifted frame: H'(i, 0) = 2 (beta - alpha), F from it
  const int gb = kBias + 2 * beta - 2 * alpha;

  for (;;) {
    int ticket = 0;
    if (t == 0) ticket = atomicAdd(&a.ctr->next_long16, 1);
    ticket = __builtin_amdgcn_readfirstlane(ticket);
    if (ticket >= n_tasks) break;
    // duo = last duo whose first task <= ticket (binary search)
    int lo = 0, hi = n_duos - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.items[2 * mid].task0 <= ticket) lo = mid;
      else hi = mid - 1;
    }
    Task T;
    const LongItem &I0 = a.items[2 * lo];
    T.d0 = I0.d;
    T.has1 = 2 * lo + 1 < n_items;
    T.d1 = PairDesc{0, 0, 0, 0, -1, 0};
    if (T.has1) T.d1 = a.items[2 * lo + 1].d;
    T.s = ticket - I0.task0;
    T.S = I0.stripes;
    T.task0 = I0.task0;
    T.bnd_off = I0.bnd_off;
    const int k = stripe_k(max(T.d0.n, T.has1 ? T.d1.n : 0), T.S);
    switch (k) {
      case 10: stripe_task<10>(a, T, rq, xq, qt, t, gb); break;
      case 11: stripe_task<11>(a, T, rq, xq, qt, t, gb); break;
      case 12: stripe_task<12>(a, T, rq, xq, qt, t, gb); break;
      case 13: stripe_task<13>(a, T, rq, xq, qt, t, gb); break;
      case 14: stripe_task<14>(a, T, rq, xq, qt, t, gb); break;
      case 15: stripe_task<15>(a, T, rq, xq, qt, t, gb); break;
      default: stripe_task<16>(a, T, rq, xq, qt, t, gb); break;
    }
  }
}

}  // namespace

int long_dp_i16_stripe_width() { return kW; }

int long_dp_i16_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, long_dp_i16_kernel, kWave, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

hipError_t launch_long_dp_i16(const Long16Args &args, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(long_dp_i16_kernel, dim3(grid), dim3(kWave), 0, stream, args);
  return hipGetLastError();
}

}  // namespace asmi
