// Per-pair features of the learned band: a histogram of the diagonals on
// which 7-mers of A meet unique 7-mers of B, plus two length/identity terms.
//
// One 256-thread workgroup per pair at a time (the grid strides over the
// pairs); thread t handles positions t, t + 256, ... of each sequence, which
// keeps many independent loads in flight.  B's 7-mers go into a direct-
// mapped LDS table of 4^7 32-bit entries (64 KB) holding
// [generation:8][duplicate:1][position + 1:16]; the generation is the pair's
// sequence number inside the workgroup (1..255), so entries left by earlier
// pairs read as empty and the table is cleared only once every 255 pairs.
// The first occurrence of a k-mer claims its entry with a compare-and-swap;
// any later one sets the duplicate bit, so the final state does not depend
// on the order of the threads.  A's 7-mers are then looked up and each hit on
// a unique entry adds one to a signed log-spaced bin of its deviation from
// the expected diagonal:
//   delta = (j - i) - trunc(i * (n - m) / m),
//   b = min(14, floor(log2(1 + |delta|))),  bin = 15 + b (delta >= 0), 14 - b.
// The expected shift is carried along a thread's positions as quotient and
// remainder of i |n - m| by m (one division per pair and thread).
// Features 0..29 are the bin counts over the number of hits, feature 30 is
// log2(1 + |n - m|) / 16 and feature 31 the hits over the m - 6 k-mers of A.
// Ratios are formed in double precision and rounded once to float.
#include "internal.h"

namespace asmi {
namespace {

constexpr int kK = 7;
constexpr int kTable = 1 << (2 * kK);
constexpr int64_t kMaxPos = 65535;  // B k-mers starting at or after this are not used
constexpr int kThreads = 256;
constexpr uint32_t kDupBit = 1u << 16;
constexpr uint32_t kPosMask = 0xFFFFu;
constexpr uint32_t kGenMask = 0xFF000000u;

__device__ __forceinline__ uint32_t kmer_at(const uint8_t *s, int64_t p, int &bad) {
  uint32_t c = 0;
#pragma unroll
  for (int t = 0; t < kK; ++t) {
    const uint32_t x = s[p + t];
    bad |= x > 3u;
    c = (c << 2) | (x & 3u);
  }
  return c;
}

__global__ void __launch_bounds__(kThreads) features_kernel(const uint8_t *seqs_a, const int64_t *offs_a,
                                                            const uint8_t *seqs_b, const int64_t *offs_b,
                                                            int64_t n_pairs, float *out, int32_t *status) {
  __shared__ uint32_t tab[kTable];
  __shared__ int hist[32];  // 30 bins, [30] = hits
  if (threadIdx.x < 32) hist[threadIdx.x] = 0;
  int bad = 0, bad_offs = 0;
  uint32_t gen = 0;
  for (int64_t p = blockIdx.x; p < n_pairs; p += gridDim.x) {
    gen = gen % 255u + 1u;  // 1..255; 0 marks an empty entry
    if (gen == 1) {         // every 255 pairs: a clean table
      __syncthreads();
      for (int i = threadIdx.x; i < kTable; i += kThreads) tab[i] = 0u;
    }
    const uint32_t tag = gen << 24;
    const int64_t a0 = offs_a[p], a1 = offs_a[p + 1], b0 = offs_b[p], b1 = offs_b[p + 1];
    if (a0 < 0 || b0 < 0 || a1 < a0 || b1 < b0) {  // uniform over the workgroup
      bad_offs = 1;
      if (threadIdx.x < 32) out[p * 32 + threadIdx.x] = 0.f;
      continue;
    }
    const int64_t m = a1 - a0, n = b1 - b0;
    const uint8_t *A = seqs_a + a0;
    const uint8_t *B = seqs_b + b0;
    __syncthreads();  // the table is clean / the previous pair's lookups are done
    // ---- B: claim entries ----
    const int64_t nb = (n - kK + 1) < kMaxPos ? (n - kK + 1) : kMaxPos;
    for (int64_t j = threadIdx.x; j < nb; j += kThreads) {
      const uint32_t c = kmer_at(B, j, bad);
      const uint32_t mine = tag | (uint32_t)(j + 1);
      uint32_t e = tab[c];
      if ((e & kGenMask) != tag) {
        const uint32_t prev = atomicCAS(&tab[c], e, mine);
        e = (prev == e) ? mine : prev;  // claimed, or someone of this pair was first
      }
      if (e != mine) atomicOr(&tab[c], kDupBit);
    }
    __syncthreads();
    // ---- A: look up ----
    const int64_t na = m - kK + 1;
    if (na > 0) {
      const int64_t dabs = n > m ? n - m : m - n;
      const int64_t step = dabs * kThreads;  // i grows by 256 per iteration
      const int64_t sq = step / m, sr = step % m;
      int64_t eq = (int64_t)threadIdx.x * dabs / m, er = (int64_t)threadIdx.x * dabs % m;
      for (int64_t i = threadIdx.x; i < na; i += kThreads) {
        const uint32_t c = kmer_at(A, i, bad);
        const uint32_t e = tab[c];
        if ((e & kGenMask) == tag && !(e & kDupBit)) {
          const int64_t j = (int64_t)(e & kPosMask) - 1;
          const int64_t delta = (j - i) - (n >= m ? eq : -eq);
          const int64_t ad = delta < 0 ? -delta : delta;
          int b = 63 - __clzll((unsigned long long)(ad + 1));
          b = b < 14 ? b : 14;
          atomicAdd(&hist[delta >= 0 ? 15 + b : 14 - b], 1);
          atomicAdd(&hist[30], 1);
        }
        eq += sq;
        er += sr;
        if (er >= m) {
          er -= m;
          ++eq;
        }
      }
    }
    __syncthreads();
    int hv = 0, hits = 0;
    if (threadIdx.x < 32) {
      hv = hist[threadIdx.x];
      hits = hist[30];
    }
    __syncthreads();
    if (threadIdx.x < 32) {
      hist[threadIdx.x] = 0;
      const int k = threadIdx.x;
      double f;
      if (k < 30) f = (double)hv / (double)(hits > 1 ? hits : 1);
      else if (k == 30) f = log2((double)(1 + (n > m ? n - m : m - n))) / 16.0;
      else f = (double)hits / (double)(m - (kK - 1) > 1 ? m - (kK - 1) : 1);
      out[p * 32 + k] = (float)f;
    }
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
