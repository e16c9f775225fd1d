// Per-pair features of the learned band: a histogram of the diagonals on
// which 7-mers of A meet unique 7-mers of B, plus two length/identity terms.
//
// One 512-thread workgroup per pair at a time (the grid strides over the
// pairs).  Each sequence is read in tiles of up to 8192 k-mer positions:
// the waves load the tile's residues with coalesced byte loads and pack
// them, 16 to a 32-bit word, into LDS as 2-bit codes (an OR across each
// 16-lane row through DPP), so a k-mer is two LDS words and one funnel
// shift.  The k-mer code is the 14-bit window with the first residue in
// the low bits: any fixed bijection serves, since only equality of k-mers
// matters.
// B's 7-mers go into a direct-mapped LDS table of 4^7 32-bit entries (64 KB)
// holding [generation:8][duplicate:1][position + 1:16]; the generation is
// the pair's sequence number inside the workgroup (1..255), so entries left
// by earlier pairs read as empty and the table is cleared only once every
// 255 pairs.  The first occurrence of a k-mer claims its entry with a
// compare-and-swap; any later one sets the duplicate bit, so the final state
// does not depend on the order of the threads.  A's 7-mers are then looked
// up and each hit on a unique entry adds one to a signed log-spaced bin of
// its deviation from the expected diagonal:
//   delta = (j - i) - trunc(i * (n - m) / m),
//   b = min(14, floor(log2(1 + |delta|))),  bin = 15 + b (delta >= 0), 14 - b.
// A wave adds its hits to the LDS histogram with one atomic per distinct bin
// (ballot over the lanes); histograms alternate between two buffers by pair
// parity so that one is cleared while the other fills.  The expected shift
// is carried along a thread's positions as quotient and remainder of
// i |n - m| by m.  The next pair's offsets are loaded ahead, and the first
// tiles of both sequences are loaded together before either is packed.
// Features 0..29 are the bin counts over the number of hits, feature 30 is
// log2(1 + |n - m|) / 16 and feature 31 the hits over the m - 6 k-mers of A.
// Ratios are formed in double precision and rounded once to float.
#include "internal.h"

namespace asmi {
namespace {

constexpr int kK = 7;
constexpr int kTable = 1 << (2 * kK);
constexpr int64_t kMaxPos = 65535;  // B k-mers starting at or after this are not used
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / kWave;
constexpr int kTile = 8192;                       // k-mer positions per staged tile
// words written by whole 64-residue segments, + one read past the last k-mer
constexpr int kTileWords = (kTile + kK - 1 + kWave - 1) / kWave * 4 + 1;
constexpr uint32_t kDupBit = 1u << 16;
constexpr uint32_t kPosMask = 0xFFFFu;
constexpr uint32_t kGenMask = 0xFF000000u;

// Residues [p0, p0 + cnt) of S as 2-bit codes: residue q at bits 2 (q & 15)
// of word q >> 4.  Wave w takes 64-residue segments w, w + kWaves, ...; all
// loads of a tile are issued first (stage_load), then packed (stage_pack).
constexpr int kSegs = (kTile + kK - 1 + kWave - 1) / kWave;
constexpr int kSegPerWave = (kSegs + kWaves - 1) / kWaves;

__device__ inline void stage_load(const uint8_t *S, int64_t p0, int cnt, uint32_t (&x)[kSegPerWave]) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int r = 0; r < kSegPerWave; ++r) {
    const int q = (wave + r * kWaves) * kWave + lane;
    x[r] = q < cnt ? (uint32_t)S[p0 + q] : 0u;
  }
}

__device__ inline void stage_pack(int cnt, const uint32_t (&x)[kSegPerWave], uint32_t *buf, int &bad) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int r = 0; r < kSegPerWave; ++r) {
    const int seg = wave + r * kWaves;
    if (seg * kWave >= cnt) break;  // uniform over the wave
    bad |= x[r] > 3u;
    uint32_t v = (x[r] & 3u) << (2 * (lane & 15));
    // prefix OR along each 16-lane row (lanes shifted in from outside the row read 0)
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
    if ((lane & 15) == 15) buf[seg * 4 + (lane >> 4)] = v;
  }
}

__device__ inline uint32_t kmer_at(const uint32_t *buf, int q) {
  const uint32_t lo = buf[q >> 4], hi = buf[(q >> 4) + 1];
  return __builtin_amdgcn_alignbit(hi, lo, 2u * (uint32_t)(q & 15)) & (uint32_t)(kTable - 1);
}

// Adds each lane's bin (b >= 0) to hist with one LDS atomic per distinct bin
// of the wave, and the number of hits to hist[30].
__device__ inline void wave_hist_add(int *hist, int b) {
  const int lane = threadIdx.x % kWave;
  uint64_t act = __builtin_amdgcn_ballot_w64(b >= 0);
  if (!act) return;
  if (lane == 0) atomicAdd(&hist[30], __popcll(act));
  while (act) {
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int bl = __builtin_amdgcn_readlane(b, leader);
    const uint64_t same = __builtin_amdgcn_ballot_w64(b == bl);
    if (lane == leader) atomicAdd(&hist[bl], __popcll(same));
    act &= ~same;
  }
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) features_kernel(const uint8_t *seqs_a, const int64_t *offs_a,
                                                            const uint8_t *seqs_b, const int64_t *offs_b,
                                                            int64_t n_pairs, float *out, int32_t *status) {
  __shared__ uint32_t tab[kTable];
  __shared__ uint32_t bufA[kTileWords], bufB[kTileWords];
  __shared__ int hist[2][32];  // per pair parity: 30 bins, [30] = hits
  if (threadIdx.x < 64) hist[threadIdx.x >> 5][threadIdx.x & 31] = 0;
  int bad = 0, bad_offs = 0;
  uint32_t gen = 0;
  int par = 0;
  // the next pair's offsets are loaded while this one is processed
  int64_t a0n = 0, a1n = 0, b0n = 0, b1n = 0;
  if (blockIdx.x < n_pairs) {
    a0n = offs_a[blockIdx.x];
    a1n = offs_a[blockIdx.x + 1];
    b0n = offs_b[blockIdx.x];
    b1n = offs_b[blockIdx.x + 1];
  }
  for (int64_t p = blockIdx.x; p < n_pairs; p += gridDim.x) {
    const int64_t a0 = a0n, a1 = a1n, b0 = b0n, b1 = b1n;
    const int64_t pn = p + gridDim.x;
    if (pn < n_pairs) {
      a0n = offs_a[pn];
      a1n = offs_a[pn + 1];
      b0n = offs_b[pn];
      b1n = offs_b[pn + 1];
    }
    gen = gen % 255u + 1u;  // 1..255; 0 marks an empty entry
    if (gen == 1) {         // every 255 pairs: a clean table
      __syncthreads();
      for (int i = threadIdx.x; i < kTable; i += kThreads) tab[i] = 0u;
    }
    const uint32_t tag = gen << 24;
    int *h = hist[par];
    if (a0 < 0 || b0 < 0 || a1 < a0 || b1 < b0) {  // uniform over the workgroup
      bad_offs = 1;
      if (threadIdx.x < 32) out[p * 32 + threadIdx.x] = 0.f;
      continue;
    }
    const int64_t m = a1 - a0, n = b1 - b0;
    const uint8_t *A = seqs_a + a0;
    const uint8_t *B = seqs_b + b0;
    const int64_t nb = (n - kK + 1) < kMaxPos ? (n - kK + 1) : kMaxPos;  // B k-mers used
    const int64_t na = m - kK + 1;                                        // A k-mers
    // first tiles of both sequences: every load in flight before packing
    {
      const int cb = nb > 0 ? (int)(nb < kTile ? nb : kTile) + kK - 1 : 0;
      const int ca = na > 0 ? (int)(na < kTile ? na : kTile) + kK - 1 : 0;
      uint32_t xb[kSegPerWave], xa[kSegPerWave];
      stage_load(B, 0, cb, xb);
      stage_load(A, 0, ca, xa);
      stage_pack(cb, xb, bufB, bad);
      stage_pack(ca, xa, bufA, bad);
    }
    // ---- B: claim entries ----
    for (int64_t j0 = 0; j0 < nb; j0 += kTile) {
      const int nk = (int)((nb - j0) < kTile ? (nb - j0) : kTile);
      if (j0 > 0) {  // B longer than one tile
        __syncthreads();
        uint32_t xb[kSegPerWave];
        stage_load(B, j0, nk + kK - 1, xb);
        stage_pack(nk + kK - 1, xb, bufB, bad);
      }
      __syncthreads();  // the table is clean, the tile is staged
      for (int q = threadIdx.x; q < nk; q += kThreads) {
        const uint32_t c = kmer_at(bufB, q);
        const uint32_t mine = tag | (uint32_t)(j0 + q + 1);
        uint32_t e = tab[c];
        if ((e & kGenMask) != tag) {
          const uint32_t prev = atomicCAS(&tab[c], e, mine);
          e = (prev == e) ? mine : prev;  // claimed, or someone of this pair was first
        }
        if (e != mine) atomicOr(&tab[c], kDupBit);
      }
    }
    __syncthreads();  // B's claims are done (and A's first tile is staged)
    // ---- A: look up ----
    if (na > 0) {
      const int64_t dabs = n > m ? n - m : m - n;
      const int64_t step = dabs * kThreads;  // i grows by kThreads per iteration
      const int64_t sq = step / m, sr = step % m;
      for (int64_t i0 = 0; i0 < na; i0 += kTile) {
        const int nk = (int)((na - i0) < kTile ? (na - i0) : kTile);
        if (i0 > 0) {  // A longer than one tile
          __syncthreads();
          uint32_t xa[kSegPerWave];
          stage_load(A, i0, nk + kK - 1, xa);
          stage_pack(nk + kK - 1, xa, bufA, bad);
          __syncthreads();
        }
        // the lookups of this tile; T = int when every position, shift and
        // shift step fits 30 bits (always in practice), else int64_t
        auto lookups = [&](auto zero) {
          using T = decltype(zero);
          const T i_first = (T)(i0 + threadIdx.x);
          T eq = (T)(((int64_t)i_first * dabs) / m), er = (T)(((int64_t)i_first * dabs) % m);
          const T tsq = (T)sq, tsr = (T)sr, tm = (T)m, ti0 = (T)i0;
          const bool wide = n >= m;
          // every lane of a wave runs the same number of iterations (the wave
          // aggregates its histogram updates); lanes past the tile add nothing
          const int iters = (nk + kThreads - 1) / kThreads;
          for (int r = 0; r < iters; ++r) {
            const int q = threadIdx.x + r * kThreads;
            int bin = -1;
            if (q < nk) {
              const uint32_t e = tab[kmer_at(bufA, q)];
              if ((e & kGenMask) == tag && !(e & kDupBit)) {
                const T j = (T)(e & kPosMask) - 1;
                const T delta = (j - (ti0 + q)) - (wide ? eq : -eq);
                const T ad = delta < 0 ? -delta : delta;
                int b = sizeof(T) == 4 ? 31 - __clz((int)(ad + 1)) : 63 - __clzll((long long)(ad + 1));
                b = b < 14 ? b : 14;
                bin = delta >= 0 ? 15 + b : 14 - b;
              }
            }
            wave_hist_add(h, bin);
            eq += tsq;
            er += tsr;
            if (er >= tm) {
              er -= tm;
              ++eq;
            }
          }
        };
        if (m < (1 << 30) && n < (1 << 30) && sq < (1 << 30)) lookups(0);
        else lookups((int64_t)0);
      }
    }
    __syncthreads();  // the histogram is complete
    if (threadIdx.x < 32) {
      const int k = threadIdx.x;
      const int hv = h[k], hits = h[30];
      hist[par ^ 1][k] = 0;  // the next pair's histogram (last read before this pair's first barrier)
      double f;
      if (k < 30) f = (double)hv / (double)(hits > 1 ? hits : 1);
      else if (k == 30) f = log2((double)(1 + (n > m ? n - m : m - n))) / 16.0;
      else f = (double)hits / (double)(m - (kK - 1) > 1 ? m - (kK - 1) : 1);
      out[p * 32 + k] = (float)f;
    }
    par ^= 1;  // (a skipped pair keeps the parity: its histogram stays clean)
  }
  if (bad) atomicOr(status, kStatusBadResidue);
  if (bad_offs && threadIdx.x == 0) atomicOr(status, kStatusBadOffsets);
}

}  // namespace

hipError_t launch_features(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                           const int64_t *offs_b, int64_t n_pairs, float *out, int32_t *status,
                           int num_cu, hipStream_t stream) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, features_kernel, kThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int64_t grid = (int64_t)per_cu * num_cu;
  if (grid > n_pairs) grid = n_pairs;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, seqs_a, offs_a,
                     seqs_b, offs_b, n_pairs, out, status);
  return hipGetLastError();
}

}  // namespace asmi
