// Long pairs: an anti-diagonal wavefront of column stripes across waves.
//
// The paper processes a long subject in l stages left to right inside one
// warp, handing the stage's right-hand column to the next stage through
// memory (section 3.1, last paragraphs).  For a few very long pairs that
// leaves most of the GPU idle, so here the stages run concurrently: a whole
// wave64 is one 64-lane systolic pipeline (DPP wave_shr:1 carries H and F
// from lane t-1 to lane t; lane 0 reads the boundary), owning 64*K columns,
// and stripe s+1 of a pair runs on another wave right behind stripe s.  The
// boundary column (H', F^ per row) goes through global memory with
// device-coherent (agent-scope) accesses: the producer's boundary stores and
// its progress counter bypass the non-coherent caches, the producer waits
// for its stores to complete (s_waitcnt) before it publishes how many rows
// are done, every 16 steps, and the consumer spins on the counter before it
// loads the rows of its next 16-step chunk, one chunk ahead.  The rows lane
// 63 finishes during a chunk are staged in LDS and stored at its end by 16
// lanes as one contiguous 128-byte block, so the device-coherent stores
// write whole cache lines instead of one partial line per row.  No L2
// write-back or invalidation is needed, which the agent-scope fences would
// issue on every hand-off.  Stripes are taken by persistent waves in ticket
// order (pair-major, stripe-minor), so a wave only ever waits for a stripe
// whose ticket was taken earlier by a wave that is already running: the
// wavefront cannot deadlock.  A bounded spin (seconds) turns any unexpected
// stall into an error status instead of a hang.
//
// Cell update, frames, padding and results are those of full_dp_i32.hip.
#include "internal.h"

namespace asmi {
namespace {

constexpr int kKL = 16;              // columns per lane
constexpr int kChunk = 16;           // rows per feed refill / publication
constexpr unsigned kSpinLimit = 1u << 25;

__device__ __forceinline__ int wave_shr1(int old, int src) {
  // wave_shr:1 -- lane t reads lane t-1; lane 0 keeps `old`
  return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int wave_shl1(int old, int src) {
  // wave_shl:1 -- lane t reads lane t+1; lane 63 keeps `old`
  return __builtin_amdgcn_update_dpp(old, src, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ int imax3(int a, int b, int c) { return max(max(a, b), c); }
__device__ __forceinline__ int wave_max(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ void store_bnd(int2 *p, int h, int f) {
  const long long v = (long long)(unsigned)h | ((long long)(unsigned)f << 32);
  __hip_atomic_store((long long *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int2 load_bnd(const int2 *p) {
  const long long v =
      __hip_atomic_load((const long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_int2((int)(unsigned)(v & 0xffffffffll), (int)(unsigned)((unsigned long long)v >> 32));
}

// Wait until the producer has published at least `need` rows.  The counter
// and the boundary rows are read with device-coherent loads; the loads of the
// rows are issued only after this loop has seen the counter.
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

// Publish `rows` complete rows: wait until every earlier store of this wave
// (the boundary rows) has completed, then store the counter.
__device__ __forceinline__ void publish_rows(int *flag, int rows) {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_store(flag, rows, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int MODE, int K>
__global__ void __launch_bounds__(kWave) long_dp_i32_kernel(LongDpArgs a) {
  constexpr int W = kWave * K;
  extern __shared__ __align__(16) int8_t lds[];
  __shared__ int2 xq[kChunk];  // the exported column of one chunk
  const int t = threadIdx.x;
  const int asz = a.asz;
  int8_t *prof = lds;
  const int alpha = a.alpha, beta = a.beta, amb = alpha - beta;
  const int bias = (MODE == kLocal) ? alpha : alpha + beta;
  const int n_tasks = a.ctr->n_long_tasks;
  const int n_items = a.ctr->n_long;

  for (;;) {
    int ticket = 0;
    if (t == 0) ticket = atomicAdd(&a.ctr->next_long, 1);
    ticket = __shfl(ticket, 0);
    if (ticket >= n_tasks) break;
    // item = last long item whose first task <= ticket (binary search)
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.items[mid].task0 <= ticket) lo = mid;
      else hi = mid - 1;
    }
    const LongItem it_ = a.items[lo];
    const PairDesc &d = it_.d;
    const int s = ticket - it_.task0;
    const int S = it_.stripes;
    const int m = d.m, n = d.n;
    const int pad = (MODE == kGlobal) ? 0 : S * W - n;
    const bool tr = (d.flags & kTransposed) != 0;
    const uint8_t *rows = (tr ? a.seqs_b : a.seqs_a) + d.row_off;
    const uint8_t *cols = (tr ? a.seqs_a : a.seqs_b) + d.col_off;
    const bool import = s > 0;
    const bool export_ = s + 1 < S;
    const int2 *bin = a.bnd + it_.bnd_off + (int64_t)(s - 1) * (m + 1);
    int2 *bout = a.bnd + it_.bnd_off + (int64_t)s * (m + 1);
    int *flag_in = a.flags + it_.task0 + s - 1;
    int *flag_out = a.flags + it_.task0 + s;
    int bad = 0;

    const int jp0 = s * W + t * K;
    // ---- profile of this lane's K columns ----
#pragma unroll
    for (int x = 0; x < K; ++x) {
      const int j = jp0 + x + 1 - pad;
      int c = -1;
      if (j >= 1 && j <= n) {
        c = cols[j - 1];
        if (c >= asz) { bad = 1; c = 0; }
      }
      for (int r = 0; r < asz; ++r) {
        int sv = 0;
        if (c >= 0) sv = tr ? a.subst[c * asz + r] : a.subst[r * asz + c];
        prof[r * W + t * K + x] = (int8_t)(sv + bias);
      }
    }
    // ---- row-0 state ----
    int Ha[K], Ee[K];
#pragma unroll
    for (int x = 0; x < K; ++x) {
      const int jp = jp0 + x + 1;
      if (MODE == kGlobal) { Ha[x] = 2 * beta - 2 * alpha; Ee[x] = kNegInf32; }
      else if (MODE == kSemiGlobal) { Ha[x] = beta * jp + beta - alpha; Ee[x] = kNegInf32; }
      else { Ha[x] = -alpha; Ee[x] = 0; }
    }
    int hl_prev;
    if (MODE == kGlobal) hl_prev = (jp0 == 0) ? beta - alpha : 2 * beta - 2 * alpha;
    else if (MODE == kSemiGlobal) hl_prev = beta * jp0 + beta - alpha;
    else hl_prev = -alpha;
    int fout = (MODE == kLocal) ? 0 : kNegInf32;
    int rm = (MODE == kSemiGlobal) ? kNegInf32 : 0;
    int rowoff = beta * (1 - t);
    int hb, fb;
    if (MODE == kGlobal) { hb = 2 * beta - 2 * alpha; fb = hb; }
    else if (MODE == kSemiGlobal) { hb = 2 * beta - alpha; fb = hb; }
    else { hb = -alpha; fb = 0; }

    const int its = m + kWave - 1;
    int seen = 0;  // rows the producer is known to have published
    int qfeed = 0, hfeed = 0, ffeed = 0, qc = 0;
    // feed of chunk it0: rows it0+1 .. it0+16 in lanes 0..15
    auto load_feed = [&](int it0, int &q, int &h, int &f) {
      if (import && it0 + 1 <= m) {
        const int need = min(it0 + kChunk, m);
        if (seen < need) seen = wait_rows(flag_in, need, &a.ctr->status);
      }
      if (t < kChunk) {
        const int qi = it0 + t;
        q = 0;
        if (qi < m) q = rows[qi];  // checked where it is used
        if (import && qi + 1 <= m) {
          const int2 v = load_bnd(bin + qi + 1);
          h = v.x;
          f = v.y;
        }
      }
    };
    // profile words of the row letter a lane works on (always a letter of
    // the alphabet, so the read stays inside the profile)
    auto load_prof = [&](int q, int (&w)[K / 4]) {
      const int8_t *pp = prof + q * W + t * K;
      if constexpr (K % 16 == 0) {
#pragma unroll
        for (int v = 0; v < K / 16; ++v) {
          const int4 r = *(const int4 *)(pp + 16 * v);
          w[4 * v] = r.x;
          w[4 * v + 1] = r.y;
          w[4 * v + 2] = r.z;
          w[4 * v + 3] = r.w;
        }
      } else {
        static_assert(K == 8, "K is 8 or a multiple of 16");
        const int2 r = *(const int2 *)pp;
        w[0] = r.x;
        w[1] = r.y;
      }
    };
    load_feed(0, qfeed, hfeed, ffeed);
    if (qfeed >= asz) { bad = 1; qfeed = 0; }
    for (int it0 = 0; it0 < its; it0 += kChunk) {
      int qnext = 0, hnext = 0, fnext = 0;
      if (it0 + kChunk < its) load_feed(it0 + kChunk, qnext, hnext, fnext);
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        const int row = it0 + u + 1 - t;
        qc = wave_shr1(qfeed, qc);
        const int hl = wave_shr1(import ? hfeed : hb, Ha[K - 1]);
        const int fl = wave_shr1(import ? ffeed : fb, fout);
        if ((unsigned)(row - 1) < (unsigned)m) {
          int pw[K / 4];
          load_prof(qc, pw);
          int tt[K];
#pragma unroll
          for (int x = 0; x < K; ++x) {
            const int sc = (int)(int8_t)(pw[x >> 2] >> (8 * (x & 3)));
            tt[x] = ((x == 0) ? hl_prev : Ha[x - 1]) + sc;
            if (MODE != kLocal) Ee[x] = max(Ee[x], Ha[x]);
          }
          int f = fl;
#pragma unroll
          for (int x = 0; x < K; ++x) {
            if (MODE == kLocal) {
              const int e = imax3(Ee[x] - beta, Ha[x], 0);
              const int h = imax3(tt[x], e, f);
              rm = max(rm, h);
              Ha[x] = h - alpha;
              Ee[x] = e;
              f = imax3(f - beta, Ha[x], 0);
            } else {
              const int h = imax3(tt[x], Ee[x], f);
              Ha[x] = h - amb;
              f = max(f, Ha[x]);
            }
          }
          fout = f;
          if (MODE == kSemiGlobal) rm = max(rm, Ha[K - 1] - rowoff);
          if (export_ && t == kWave - 1) xq[u] = make_int2(Ha[K - 1], fout);
        }
        hl_prev = hl;
        if (MODE == kSemiGlobal) { hb += beta; fb = hb; }
        rowoff += beta;
        qfeed = wave_shl1(qfeed, qfeed);
        hfeed = wave_shl1(hfeed, hfeed);
        ffeed = wave_shl1(ffeed, ffeed);
      }
      if (qnext >= asz) { bad = 1; qnext = 0; }
      qfeed = qnext;
      hfeed = hnext;
      ffeed = fnext;
      if (export_) {
        // lane u stores the row lane 63 finished at step it0 + u; then every
        // complete row is published
        __builtin_amdgcn_wave_barrier();
        if (t < kChunk) {
          const int row = it0 + t - (kWave - 2);
          if (row >= 1 && row <= m) {
            const int2 v = xq[t];
            store_bnd(bout + row, v.x, v.y);
          }
        }
        __builtin_amdgcn_wave_barrier();
        const int done = min(it0 + kChunk - (kWave - 1), m);
        if (done > 0) publish_rows(flag_out, done);
      }
    }
    if (export_) publish_rows(flag_out, m);

    // ---- this stripe's contribution to the pair's score ----
    int32_t *out = a.scores + d.pair;
    if (MODE == kLocal) {
      const int v = wave_max(rm);
      if (t == 0) atomicMax(out, v);
    } else if (MODE == kSemiGlobal) {
      int lr = kNegInf32;
#pragma unroll
      for (int x = 0; x < K; ++x) lr = max(lr, Ha[x] - beta * (jp0 + x + 1));
      int cand = lr + amb - beta * m;
      if (s + 1 == S && t == kWave - 1) cand = max(cand, rm + amb - beta * (S * W));
      const int v = wave_max(cand);
      if (t == 0) atomicMax(out, v);
    } else {
      const int c = n - 1 - s * W;
      int v = kNegInf32;
      if (c >= 0 && c < W && c / K == t) {
        const int xr = c % K;
#pragma unroll
        for (int x = 0; x < K; ++x) if (x == xr) v = Ha[x];
        v = v + amb - beta * (m + n);
      }
      v = wave_max(v);
      if (c >= 0 && c < W && t == 0) *out = v;
    }
    if (bad) atomicOr(&a.ctr->status, kStatusBadResidue);
  }
}

// Every alphabet takes 1024-column stripes (K = 16).  512-column stripes
// (K = 8) halve a 20-letter profile's LDS (10 KB per wave, 16 waves per CU
// instead of 8) but double the stripes and hand-offs; on 65,536-residue
// protein pairs they measured 3% slower.
constexpr int stripe_k(int) { return kKL; }

template <int MODE>
hipError_t launch_mode(const LongDpArgs &args, int grid, hipStream_t stream) {
  hipLaunchKernelGGL((long_dp_i32_kernel<MODE, kKL>), dim3(grid), dim3(kWave), long_dp_i32_lds_bytes(args.asz),
                     stream, args);
  return hipGetLastError();
}

template <int MODE>
int occupancy(size_t lds) {
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, long_dp_i32_kernel<MODE, kKL>, kWave, lds);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace

size_t long_dp_i32_lds_bytes(int asz) { return (size_t)asz * kWave * stripe_k(asz); }
int long_dp_i32_stripe_width(int asz) { return kWave * stripe_k(asz); }

int long_dp_i32_blocks_per_cu(int mode, int asz) {
  const size_t lds = long_dp_i32_lds_bytes(asz);
  if (mode == kGlobal) return occupancy<kGlobal>(lds);
  if (mode == kSemiGlobal) return occupancy<kSemiGlobal>(lds);
  return occupancy<kLocal>(lds);
}

hipError_t launch_long_dp_i32(int mode, const LongDpArgs &args, int grid, hipStream_t stream) {
  switch (mode) {
    case kGlobal: return launch_mode<kGlobal>(args, grid, stream);
    case kSemiGlobal: return launch_mode<kSemiGlobal>(args, grid, stream);
    default: return launch_mode<kLocal>(args, grid, stream);
  }
}

}  // namespace asmi
