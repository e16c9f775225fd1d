// Full Gotoh DP with 32-bit cells, one 16-lane DPP row per alignment.
//
// Method: paper section 3.1 ("Mapping Matrix Cells and Sequences to
// Threads"): lane t of a group owns K adjacent columns; in wavefront step
// `it` it computes its K cells of row it + 1 - t from registers only, takes
// the rightmost H (and F) of lane t-1 with a one-lane shift, and looks the
// substitution scores up in a per-lane scoring profile.  On gfx950 the shift
// is a DPP row_shr:1 (a VALU source modifier, no LDS traffic), the group is
// one 16-lane DPP row, and the profile is int8 in LDS.  Columns wider than
// 16*K are processed in stripes left to right with the stripe's right-hand
// H/F column written to a global boundary buffer and read back by the next
// stripe (the paper's multi-stage scheme for long subjects).
//
// Cell recurrences (paper Eq. (1),(4),(5)) are evaluated in two frames:
//
//  * global and semi-global use the shifted frame X^(i,j) = X(i,j) + beta*(i+j)
//    for X in {H, E, F}.  In it the extension penalty disappears:
//        E^(i,j)   = max(E^(i-1,j), H'(i-1,j))
//        F^(i,j+1) = max(F^(i,j),   H'(i,j))
//        H^(i,j)   = max(H'(i-1,j-1) + sigma + alpha + beta, E^(i,j), F^(i,j))
//        H'(i,j)   = H^(i,j) - (alpha - beta)
//    five VALU operations per cell (max, add, max3, sub, max) instead of the
//    paper's seven; the frame is exact integer arithmetic, undone on output.
//  * local keeps the plain frame, with E and F clamped at 0 so that the
//    nu = 0 term folds into their max3:  E'(i,j) = max(E'(i-1,j) - beta,
//    H(i-1,j) - alpha, 0), likewise F'; H = max3(H(i-1,j-1) + sigma, E', F')
//    equals max(..., E, F, 0) because E' = max(E, 0).  Seven operations per
//    cell plus the running maximum.
//
// Variants: K = 8, 16 or 32 columns per lane (stripes of 128, 256 or 512
// columns).  One persistent launch drains a work list ordered by length bin;
// the list is laid out in quads (one per wave, one item per group) that never
// mix variants, and each quad carries its K in the descriptor flags, so a
// wave takes the matching code path for all four of its groups.  The kernel
// is instantiated for the set of variants the list holds.
//
// Padding: global pads the last stripe on the right (result cell H(m,n) is
// picked out at the end).  Semi-global and local pad the first stripe on the
// left with columns whose sigma is 0: such columns keep H = 0 in every row,
// exactly the boundary column H(i,0) = 0 of these modes, and F flowing out of
// them equals H(i,0) - alpha.  Column n then sits in the last register of the
// last lane, which makes the semi-global last-column maximum one max per step.
#include "internal.h"

namespace asmi {
namespace {


__device__ __forceinline__ int dpp_shr1(int old, int src) {
  // row_shr:1 -- lane t reads lane t-1 of its 16-lane row; lane 0 keeps `old`.
  return __builtin_amdgcn_update_dpp(old, src, 0x111, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_shl1(int old, int src) {
  // row_shl:1 -- lane t reads lane t+1 of its row; lane 15 keeps `old`.
  return __builtin_amdgcn_update_dpp(old, src, 0x101, 0xF, 0xF, false);
}
__device__ __forceinline__ int imax3(int a, int b, int c) { return max(max(a, b), c); }

// LDS bytes of the profiles of a variant set (an instantiation's KMASK):
// four groups of asz rows of 16 K columns for the 32-bit variants, four
// groups of two (asz + 1)-row profiles of 128 columns for kVarP16; the mixed
// sets take the larger.
__host__ __device__ constexpr size_t full_dp_i32_profile_bytes(int asz, int inst) {
  const size_t kmax = (inst & 4) ? 32 : ((inst & 2) ? 16 : 8);
  const size_t b32 = (inst & 7) ? (size_t)kGroupsPerWave * asz * kGroup * kmax : 0;
  const size_t bp = (inst & 8) ? (size_t)kGroupsPerWave * 2 * (asz + 1) * kGroup * 8 : 0;
  return ((b32 > bp ? b32 : bp) + 15) / 16 * 16;
}

// Packed 16-bit helpers of the kVarP16 variant (two pairs per register).
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
  return __builtin_bit_cast(s2, __builtin_elementwise_sub_sat(__builtin_bit_cast(u2, a), __builtin_bit_cast(u2, b)));
}
__device__ __forceinline__ s2 group_max2(s2 v) {
  v = vmax(v, as_s2(__shfl_xor(as_i(v), 8, 16)));
  v = vmax(v, as_s2(__shfl_xor(as_i(v), 4, 16)));
  v = vmax(v, as_s2(__shfl_xor(as_i(v), 2, 16)));
  v = vmax(v, as_s2(__shfl_xor(as_i(v), 1, 16)));
  return v;
}

__device__ __forceinline__ int group_max(int v) {
  v = max(v, __shfl_xor(v, 8, 16));
  v = max(v, __shfl_xor(v, 4, 16));
  v = max(v, __shfl_xor(v, 2, 16));
  v = max(v, __shfl_xor(v, 1, 16));
  return v;
}
__device__ __forceinline__ int wave_max_groups(int v) {
  // v is uniform inside each group: combine the four groups.
  v = max(v, __shfl_xor(v, 16));
  v = max(v, __shfl_xor(v, 32));
  return v;
}

// Profile bytes of one lane's K columns for rows 0..asz-1: row r, column x
// holds tb[c[x] * asz + r], where tb is the workgroup's LDS score table of
// the pair's orientation (column letter c, row letter r; c == asz is a
// padding column, c == asz + 1 a column past the pair's stripes).  Four
// columns go out as one 32-bit LDS store.
template <int K>
__device__ __forceinline__ void write_profile(int8_t *pp, int W, const int8_t *tb, const int (&c)[K], int asz) {
  for (int r = 0; r < asz; ++r) {
#pragma unroll
    for (int x4 = 0; x4 < K / 4; ++x4) {
      uint32_t w = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) w |= (uint32_t)(uint8_t)tb[c[4 * x4 + b] * asz + r] << (8 * b);
      *(uint32_t *)(pp + r * W + 4 * x4) = w;
    }
  }
}

// One quad of items (one per group) with K columns per lane.
template <int MODE, int K>
__device__ __forceinline__ void align_quad(const FullDpArgs &a, int8_t *prof, const int8_t *stab, int2 *slot,
                                           PairDesc d, bool has, int t) {
  constexpr int W = kGroup * K;
  const int asz = a.asz;
  const int alpha = a.alpha, beta = a.beta;
  const int amb = alpha - beta;
  {
    const int m = has ? d.m : 0;
    const int n = has ? d.n : 0;
    const int S = has ? (n + W - 1) / W : 0;
    const int pad = (MODE == kGlobal) ? 0 : S * W - n;
    const bool tr = (d.flags & kTransposed) != 0;
    const uint8_t *rows = (tr ? a.seqs_b : a.seqs_a) + d.row_off;
    const uint8_t *cols = (tr ? a.seqs_a : a.seqs_b) + d.col_off;
    const int S_max = wave_max_groups(S);
    int result = 0;       // semi-global / local: boundary cells and the empty alignment give 0
    int bad = 0;          // residue codes out of range seen by this lane

    for (int s = 0; s < S_max; ++s) {
      const bool on = s < S;
      const int m_s = on ? m : 0;
      const int jp0 = s * W + t * K;   // padded column of x = 0 is jp0 + 1
      // ---- scoring profile for this lane's K columns (paper: init_profile) ----
      if (on) {
        int cc[K];  // column codes: a letter, or asz for a padding column (sigma 0, see header)
#pragma unroll
        for (int x = 0; x < K; ++x) {
          const int j = jp0 + x + 1 - pad;  // real column, 1-based
          cc[x] = asz;
          if (j >= 1 && j <= n) {
            cc[x] = cols[j - 1];
            if (cc[x] >= asz) { bad = 1; cc[x] = 0; }
          }
        }
        write_profile<K>(prof + t * K, W, stab + (tr ? (asz + 2) * asz : 0), cc, asz);
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
      int hout = Ha[K - 1];
      int fout = (MODE == kLocal) ? 0 : kNegInf32;
      int rm = 0;                 // local running max / semi-global last-column max
      if (MODE == kSemiGlobal) rm = kNegInf32;
      int rowoff = 0;             // beta * row, semi-global only

      const bool import = s > 0;
      const bool export_ = on && (s + 1 < S);
      const int2 *bin = slot + (int64_t)(s & 1) * a.bnd_rows;
      int2 *bout = slot + (int64_t)((s + 1) & 1) * a.bnd_rows;

      const int its = m_s > 0 ? m_s + kGroup - 1 : 0;
      const int its_max = wave_max_groups(its);

      // left boundary of stripe 0 for lane 0 (rows advance by one per step)
      int hb, fb;
      if (MODE == kGlobal) { hb = 2 * beta - 2 * alpha; fb = hb; }
      else if (MODE == kSemiGlobal) { hb = 2 * beta - alpha; fb = hb; }  // row 1
      else { hb = -alpha; fb = 0; }

      // feeds: query residues (and imported boundary) for 16 steps, lane t = step t
      int qfeed = 0, hfeed = 0, ffeed = 0, qc = 0;
      {
        const int qi = t;
        if (qi < m_s) { qfeed = rows[qi]; if (qfeed >= asz) { bad = 1; qfeed = 0; } }
        if (import && t + 1 <= m_s) { const int2 v = bin[t + 1]; hfeed = v.x; ffeed = v.y; }
      }
      if (MODE == kSemiGlobal) rowoff = beta * (1 - t);

      // profile words of a lane's row letter (always a letter of the
      // alphabet, so the read stays inside the profile); the letter and
      // words of step u + 1 are fetched during step u, so the LDS latency
      // overlaps a step's arithmetic
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
          static_assert(K == 8, "K is 8, 16 or 32");
          const int2 r = *(const int2 *)pp;
          w[0] = r.x;
          w[1] = r.y;
        }
      };
      qc = dpp_shr1(qfeed, qc);
      int pw[K / 4];
      load_prof(qc, pw);

      for (int it0 = 0; it0 < its_max; it0 += kGroup) {
        // the next chunk's feed; the residue is checked only where it is
        // used (the chunk's last step), so the load's latency overlaps the
        // chunk instead of stalling its start
        int qnext = 0, hnext = 0, fnext = 0;
        {
          const int qi = it0 + kGroup + t;
          if (qi < m_s) qnext = rows[qi];
          const int bi = it0 + kGroup + 1 + t;
          if (import && bi <= m_s) { const int2 v = bin[bi]; hnext = v.x; fnext = v.y; }
        }
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
          const int row = it0 + u + 1 - t;
          if (u == kGroup - 1 && qnext >= asz) { bad = 1; qnext = 0; }
          const int qf_next = (u == kGroup - 1) ? qnext : dpp_shl1(qfeed, qfeed);
          const int qc_next = dpp_shr1(qf_next, qc);
          int pw_next[K / 4];
          load_prof(qc_next, pw_next);
          const int hsrc = import ? hfeed : hb;
          const int fsrc = import ? ffeed : fb;
          const int hl = dpp_shr1(hsrc, hout);
          const int fl = dpp_shr1(fsrc, fout);
          if ((unsigned)(row - 1) < (unsigned)m_s) {
            int dg = hl_prev;
            int f = fl;
#pragma unroll
            for (int x = 0; x < K; ++x) {
              const int sc = (int)(int8_t)(pw[x >> 2] >> (8 * (x & 3)));
              if (MODE == kLocal) {
                const int e = imax3(Ee[x] - beta, Ha[x], 0);
                const int h = imax3(dg + sc, e, f);
                rm = max(rm, h);
                dg = Ha[x];
                Ha[x] = h - alpha;
                Ee[x] = e;
                f = imax3(f - beta, Ha[x], 0);
              } else {
                const int e = max(Ee[x], Ha[x]);
                const int h = imax3(dg + sc, e, f);
                dg = Ha[x];
                Ha[x] = h - amb;
                Ee[x] = e;
                f = max(f, Ha[x]);
              }
            }
            hout = Ha[K - 1];
            fout = f;
            if (MODE == kSemiGlobal) rm = max(rm, hout - rowoff);
            if (export_ && t == kGroup - 1) bout[row] = make_int2(hout, fout);
          }
          hl_prev = hl;
          if (MODE == kSemiGlobal) { hb += beta; fb = hb; rowoff += beta; }
          qfeed = qf_next;
          qc = qc_next;
#pragma unroll
          for (int v = 0; v < K / 4; ++v) pw[v] = pw_next[v];
          if (import) { hfeed = dpp_shl1(hfeed, hfeed); ffeed = dpp_shl1(ffeed, ffeed); }
        }
        qfeed = qnext;
        hfeed = hnext;
        ffeed = fnext;
      }

      // ---- per-stripe results ----
      if (MODE == kLocal) {
        result = max(result, group_max(rm));
      } else if (MODE == kSemiGlobal) {
        // last row: H(m, jp) = H'(m, jp) + alpha - beta - beta*(m + jp)
        int lr = kNegInf32;
#pragma unroll
        for (int x = 0; x < K; ++x) lr = max(lr, Ha[x] - beta * (jp0 + x + 1));
        int cand = m_s > 0 ? lr + amb - beta * m_s : kNegInf32;
        if (on && s + 1 == S && t == kGroup - 1 && m_s > 0)   // last column (jp = S*W)
          cand = max(cand, rm + amb - beta * (S * W));
        const int gm = group_max(cand);
        if (on) result = max(result, gm);
      } else {
        // H(m, n) sits in stripe (n-1)/W, lane ((n-1)%W)/K, register (n-1)%K
        const int c = n - 1 - s * W;
        int v = kNegInf32;
        if (on && c >= 0 && c < W && c / K == t) {
          const int xr = c % K;
#pragma unroll
          for (int x = 0; x < K; ++x) if (x == xr) v = Ha[x];
          v = v + amb - beta * (m + n);
        }
        v = group_max(v);
        if (on && c >= 0 && c < W) result = v;
      }
      if (s + 1 < S_max) __threadfence();  // boundary writes visible to the next stripe's loads
    }
    if (bad) atomicOr(&a.ctr->status, kStatusBadResidue);
    if (has && t == 0) a.scores[d.pair] = result;
  }
}

// kVarP16 (local mode only): the pairs d0 and d1 of one group in the low and
// high 16-bit halves of every register, K = 8 columns per lane, stripes of
// 128 columns.  Each half has its own int8 profile in LDS (asz + 1 rows of
// sigma + alpha per column; row asz is 0, the score of rows past a half's
// length, which only lowers cells), read with one 8-byte load per half and
// step; one v_perm_b32 per cell pair zero-extends the two halves' bytes
// into a packed pair.  The recurrences are those of the packed local kernel
// (full_dp_i16x2.hip): H - alpha stored, E and F clamped at 0 by unsigned
// saturating subtraction, signed saturating diagonal sums; a half whose
// maximum reaches sat_limit is queued for the 32-bit re-run.  Padding
// columns (left of stripe 0) score sigma = 0, which reproduces the boundary
// column H(i, 0) = 0; the stripes past a half's own count score 0 for every
// letter.  The boundary column carries both halves' (H - alpha, F) packed.
template <int MODE>
__device__ __forceinline__ void align_octet(const FullDpArgs &a, int8_t *prof, const int8_t *stab, int2 *slot,
                                            PairDesc d0, bool has0, PairDesc d1, bool has1, int t) {
  if constexpr (MODE != kLocal) {
    return;
  } else {
    constexpr int K = 8;
    constexpr int W = kGroup * K;
    const int asz = a.asz;
    const int alpha = a.alpha, beta = a.beta;
    const s2 alpha2 = pk(alpha, alpha), beta2 = pk(beta, beta);
    const int m0 = has0 ? d0.m : 0, m1 = has1 ? d1.m : 0;
    const int n0 = has0 ? d0.n : 0, n1 = has1 ? d1.n : 0;
    const int S0 = (n0 + W - 1) / W, S1 = (n1 + W - 1) / W;
    const int pad0 = S0 * W - n0, pad1 = S1 * W - n1;
    const bool tr0 = (d0.flags & kTransposed) != 0, tr1 = (d1.flags & kTransposed) != 0;
    const uint8_t *rows0 = (tr0 ? a.seqs_b : a.seqs_a) + d0.row_off;
    const uint8_t *cols0 = (tr0 ? a.seqs_a : a.seqs_b) + d0.col_off;
    const uint8_t *rows1 = (tr1 ? a.seqs_b : a.seqs_a) + d1.row_off;
    const uint8_t *cols1 = (tr1 ? a.seqs_a : a.seqs_b) + d1.col_off;
    const int S = max(S0, S1);
    const int S_max = wave_max_groups(S);
    const int mmax = max(m0, m1);
    int8_t *prof0 = prof, *prof1 = prof + (asz + 1) * W;
    s2 rm = pk(0, 0);
    int bad = 0;
    for (int s = 0; s < S_max; ++s) {
      const bool on = s < S;
      const int m_s = on ? mmax : 0;
      const int jp0 = s * W + t * K;
      // ---- the two profiles of this lane's K columns ----
      if (on) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int n = h ? n1 : n0, pad = h ? pad1 : pad0, Sh = h ? S1 : S0;
          const uint8_t *cols = h ? cols1 : cols0;
          const bool tr = h ? tr1 : tr0;
          int8_t *pp = (h ? prof1 : prof0) + t * K;
          // column codes: a letter, asz for a padding column (sigma 0), asz + 1
          // past the half's stripes (score 0)
          int cc[K];
#pragma unroll
          for (int x = 0; x < K; ++x) {
            const int j = jp0 + x + 1 - pad;  // real column, 1-based
            cc[x] = (s >= Sh) ? asz + 1 : asz;
            if (s < Sh && j >= 1 && j <= n) {
              cc[x] = cols[j - 1];
              if (cc[x] >= asz) { bad = 1; cc[x] = 0; }
            }
          }
          write_profile<K>(pp, W, stab + (tr ? (asz + 2) * asz : 0), cc, asz);
#pragma unroll
          for (int x4 = 0; x4 < K / 4; ++x4) *(uint32_t *)(pp + asz * W + 4 * x4) = 0u;  // the no-row row
        }
      }
      // ---- row-0 state (local: H(0, j) - alpha = -alpha, E' = 0) ----
      s2 Ha[K], Ee[K];
#pragma unroll
      for (int x = 0; x < K; ++x) {
        Ha[x] = pk(-alpha, -alpha);
        Ee[x] = pk(0, 0);
      }
      s2 hl_prev = pk(-alpha, -alpha);
      int hout = as_i(Ha[K - 1]);
      int fout = 0;
      const bool import = s > 0;
      const bool export_ = on && (s + 1 < S);
      const int2 *bin = slot + (int64_t)(s & 1) * a.bnd_rows;
      int2 *bout = slot + (int64_t)((s + 1) & 1) * a.bnd_rows;
      const int its = m_s > 0 ? m_s + kGroup - 1 : 0;
      const int its_max = wave_max_groups(its);
      const int hb = as_i(pk(-alpha, -alpha)), fb = 0;  // stripe 0's left boundary
      // feeds: the row letters of both halves (q0 | q1 << 8) and the imported
      // boundary, lane t holding step t of the chunk.  The residue bytes are
      // loaded a chunk ahead (-1: past the half's rows) and checked and
      // packed only where used, so the loads overlap the chunk.
      auto pack_rows = [&](int r0, int r1) {
        int q0 = r0 < 0 ? asz : r0, q1 = r1 < 0 ? asz : r1;
        if (r0 >= asz) { bad = 1; q0 = 0; }
        if (r1 >= asz) { bad = 1; q1 = 0; }
        return q0 | (q1 << 8);
      };
      int qfeed = 0, hfeed = 0, ffeed = 0, qc = 0;
      if (t < m_s) qfeed = pack_rows(t < m0 ? (int)rows0[t] : -1, t < m1 ? (int)rows1[t] : -1);
      if (import && t + 1 <= m_s) {
        const int2 v = bin[t + 1];
        hfeed = v.x;
        ffeed = v.y;
      }
      // The row letters and profile words of step u + 1 are fetched during
      // step u, so the LDS latency overlaps a step's arithmetic.  Letters are
      // always 0..asz (asz: the zero row), so the reads stay in the profiles.
      qc = dpp_shr1(qfeed, qc);
      int2 w0 = *(const int2 *)(prof0 + (qc & 0xFF) * W + t * K);
      int2 w1 = *(const int2 *)(prof1 + (qc >> 8) * W + t * K);
      for (int it0 = 0; it0 < its_max; it0 += kGroup) {
        int qnext = 0, hnext = 0, fnext = 0;
        const int qi = it0 + kGroup + t;
        const int nr0 = (qi < m_s && qi < m0) ? (int)rows0[qi] : -1;
        const int nr1 = (qi < m_s && qi < m1) ? (int)rows1[qi] : -1;
        {
          const int bi = it0 + kGroup + 1 + t;
          if (import && bi <= m_s) {
            const int2 v = bin[bi];
            hnext = v.x;
            fnext = v.y;
          }
        }
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
          const int row = it0 + u + 1 - t;
          if (u == kGroup - 1 && qi < m_s) qnext = pack_rows(nr0, nr1);
          const int qf_next = (u == kGroup - 1) ? qnext : dpp_shl1(qfeed, qfeed);
          const int qc_next = dpp_shr1(qf_next, qc);
          const int2 w0n = *(const int2 *)(prof0 + (qc_next & 0xFF) * W + t * K);
          const int2 w1n = *(const int2 *)(prof1 + (qc_next >> 8) * W + t * K);
          const s2 hl = as_s2(dpp_shr1(import ? hfeed : hb, hout));
          const int fl = dpp_shr1(import ? ffeed : fb, fout);
          if ((unsigned)(row - 1) < (unsigned)m_s) {
            s2 tt[K];
#pragma unroll
            for (int x = 0; x < K; ++x) {
              // bytes x & 3 of the two halves' words, zero-extended into a packed pair
              const uint32_t sel = (uint32_t)(x & 3) | 0x0C00u | ((uint32_t)(4 + (x & 3)) << 16) | 0x0C000000u;
              const s2 p = as_s2((int)__builtin_amdgcn_perm((uint32_t)(x < 4 ? w1.x : w1.y),
                                                            (uint32_t)(x < 4 ? w0.x : w0.y), sel));
              const s2 dg = (x == 0) ? hl_prev : Ha[x - 1];
              tt[x] = __builtin_elementwise_add_sat(dg, p);
            }
            s2 f = as_s2(fl);
#pragma unroll
            for (int x = 0; x < K; ++x) {
              const s2 h = vmax(vmax(tt[x], Ee[x]), f);
              rm = vmax(rm, h);
              Ha[x] = h - alpha2;
              Ee[x] = vmax(sat_sub_u(Ee[x], beta2), Ha[x]);
              f = vmax(sat_sub_u(f, beta2), Ha[x]);
            }
            hout = as_i(Ha[K - 1]);
            fout = as_i(f);
            if (export_ && t == kGroup - 1) bout[row] = make_int2(hout, fout);
          }
          hl_prev = hl;
          qfeed = qf_next;
          qc = qc_next;
          w0 = w0n;
          w1 = w1n;
          if (import) {
            hfeed = dpp_shl1(hfeed, hfeed);
            ffeed = dpp_shl1(ffeed, ffeed);
          }
        }
        qfeed = qnext;
        hfeed = hnext;
        ffeed = fnext;
      }
      if (s + 1 < S_max) __threadfence();  // boundary writes visible to the next stripe's loads
    }
    const s2 gm = group_max2(rm);
    if (bad) atomicOr(&a.ctr->status, kStatusBadResidue);
    if (t == 0) {
      if (has0) {
        if (gm.x >= a.sat_limit) a.rerun[atomicAdd(a.n_rerun, 1)] = d0;
        else a.scores[d0.pair] = gm.x;
      }
      if (has1) {
        if (gm.y >= a.sat_limit) a.rerun[atomicAdd(a.n_rerun, 1)] = d1;
        else a.scores[d1.pair] = gm.y;
      }
    }
  }
}

// Persistent kernel over the 32-bit list, claimed in units of kClaim32
// items.  KMASK is the set of variants the list may hold (bit 0: K = 8,
// bit 1: K = 16, bit 2: K = 32, bit 3: packed kVarP16); a single-variant
// instantiation has no dispatch and the register footprint of that variant
// alone, the mixed ones size registers and LDS for the widest.  A unit of a
// 32-bit variant is two quads (one item per group each, run one after the
// other); a kVarP16 unit is one octet (two items per group, run together).
template <int MODE, int KMASK>
__global__ void __launch_bounds__(kWave) full_dp_i32_kernel(FullDpArgs a) {
  constexpr int KMAX = (KMASK & 4) ? 32 : ((KMASK & 2) ? 16 : 8);
  constexpr bool HAS32 = (KMASK & 7) != 0, HASP = (KMASK & 8) != 0;
  extern __shared__ __align__(16) int8_t lds[];
  const int lane = threadIdx.x;
  const int g = lane >> 4;
  const int t = lane & 15;
  int8_t *prof = lds + g * a.asz * (kGroup * KMAX);
  int8_t *prof_p = lds + g * 2 * (a.asz + 1) * (kGroup * 8);
  // Score table after the profiles, filled once per workgroup: orientation o
  // (1: the pair is transposed), column code c, row letter r ->
  // sigma(r, c) + bias (o = 0) or sigma(c, r) + bias (o = 1) for letters,
  // the bias for c = asz (padding column, sigma 0), 0 for c = asz + 1.
  int8_t *stab = lds + full_dp_i32_profile_bytes(a.asz, KMASK);
  {
    const int asz = a.asz, tn = (asz + 2) * asz;
    const int bias = (MODE == kLocal) ? a.alpha : a.alpha + a.beta;
    for (int i = lane; i < 2 * tn; i += kWave) {
      const int o = i >= tn ? 1 : 0, k = i - o * tn, c = k / asz, r = k - c * asz;
      int v = 0;
      if (c < asz) v = (o ? a.subst[c * asz + r] : a.subst[r * asz + c]) + bias;
      else if (c == asz) v = bias;
      stab[i] = (int8_t)v;
    }
    __syncthreads();
  }
  const int n_items = *a.n_items;
  int2 *slot = a.bnd + ((int64_t)blockIdx.x * kGroupsPerWave + g) * 2 * a.bnd_rows;
  for (;;) {
    int base = 0;
    if (lane == 0) base = atomicAdd(a.next, kClaim32);
    base = __shfl(base, 0);
    if (base >= n_items) break;
    // the unit's variant (units never mix variants)
    int kv = 0;
    if (lane == 0) kv = variant_of(a.items[base].flags);
    kv = __shfl(kv, 0);
    bool octet = false;
    if constexpr (HASP) octet = !HAS32 || kv == kVarP16;
    if (octet) {
      if constexpr (HASP) {
        const int i0 = base + 2 * g, i1 = i0 + 1;
        PairDesc d0{0, 0, 0, 0, -1, 0}, d1{0, 0, 0, 0, -1, 0};
        if (i0 < n_items) d0 = a.items[i0];
        if (i1 < n_items) d1 = a.items[i1];
        align_octet<MODE>(a, prof_p, stab, slot, d0, i0 < n_items && d0.pair >= 0, d1,
                          i1 < n_items && d1.pair >= 0, t);
      }
    } else {
      if constexpr (HAS32) {
        for (int q = 0; q < kClaim32 / kGroupsPerWave; ++q) {
          const int item = base + q * kGroupsPerWave + g;
          PairDesc d{0, 0, 0, 0, -1, 0};
          if (item < n_items) d = a.items[item];
          const bool has = item < n_items && d.pair >= 0;  // padding slots carry pair -1
          if constexpr ((KMASK & 7) == 1) {
            align_quad<MODE, 8>(a, prof, stab, slot, d, has, t);
          } else if constexpr ((KMASK & 7) == 2) {
            align_quad<MODE, 16>(a, prof, stab, slot, d, has, t);
          } else if constexpr ((KMASK & 7) == 4) {
            align_quad<MODE, 32>(a, prof, stab, slot, d, has, t);
          } else {
            if (kv == kVarI32K8) align_quad<MODE, 8>(a, prof, stab, slot, d, has, t);
            else if (kv == kVarI32K32) align_quad<MODE, 32>(a, prof, stab, slot, d, has, t);
            else align_quad<MODE, 16>(a, prof, stab, slot, d, has, t);
          }
        }
      }
    }
  }
}

// The instantiation covering a set of variants: one of them alone, all
// 32-bit ones, or everything.
int kmask_instance(int kmask) {
  if (kmask == 1 || kmask == 2 || kmask == 4 || kmask == 8) return kmask;
  return (kmask & 8) ? 15 : 7;
}

template <int MODE>
hipError_t launch_mode(const FullDpArgs &args, int kmask, int grid, hipStream_t stream) {
  const size_t lds = full_dp_i32_lds_bytes(args.asz, kmask);
  switch (kmask_instance(kmask)) {
    case 1: hipLaunchKernelGGL((full_dp_i32_kernel<MODE, 1>), dim3(grid), dim3(kWave), lds, stream, args); break;
    case 2: hipLaunchKernelGGL((full_dp_i32_kernel<MODE, 2>), dim3(grid), dim3(kWave), lds, stream, args); break;
    case 4: hipLaunchKernelGGL((full_dp_i32_kernel<MODE, 4>), dim3(grid), dim3(kWave), lds, stream, args); break;
    case 8: hipLaunchKernelGGL((full_dp_i32_kernel<MODE, 8>), dim3(grid), dim3(kWave), lds, stream, args); break;
    case 15: hipLaunchKernelGGL((full_dp_i32_kernel<MODE, 15>), dim3(grid), dim3(kWave), lds, stream, args); break;
    default: hipLaunchKernelGGL((full_dp_i32_kernel<MODE, 7>), dim3(grid), dim3(kWave), lds, stream, args); break;
  }
  return hipGetLastError();
}

template <int MODE, int KMASK>
int occupancy(size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, full_dp_i32_kernel<MODE, KMASK>, kWave, lds) !=
          hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

template <int MODE>
int occupancy_mode(int kmask, size_t lds) {
  switch (kmask_instance(kmask)) {
    case 1: return occupancy<MODE, 1>(lds);
    case 2: return occupancy<MODE, 2>(lds);
    case 4: return occupancy<MODE, 4>(lds);
    case 8: return occupancy<MODE, 8>(lds);
    case 15: return occupancy<MODE, 15>(lds);
    default: return occupancy<MODE, 7>(lds);
  }
}

}  // namespace

size_t full_dp_i32_lds_bytes(int asz, int kmask) {
  // profiles, then the score table (two orientations of (asz + 2) x asz bytes)
  const size_t tab = ((size_t)2 * (asz + 2) * asz + 15) / 16 * 16;
  return full_dp_i32_profile_bytes(asz, kmask_instance(kmask)) + tab;
}
int full_dp_i32_stripe_width(int k) { return kGroup * k; }

int full_dp_i32_blocks_per_cu(int mode, int asz, int kmask) {
  const size_t lds = full_dp_i32_lds_bytes(asz, kmask);
  if (mode == kGlobal) return occupancy_mode<kGlobal>(kmask, lds);
  if (mode == kSemiGlobal) return occupancy_mode<kSemiGlobal>(kmask, lds);
  return occupancy_mode<kLocal>(kmask, lds);
}

hipError_t launch_full_dp_i32(int mode, const FullDpArgs &args, int kmask, int grid, hipStream_t stream) {
  switch (mode) {
    case kGlobal: return launch_mode<kGlobal>(args, kmask, grid, stream);
    case kSemiGlobal: return launch_mode<kSemiGlobal>(args, kmask, grid, stream);
    default: return launch_mode<kLocal>(args, kmask, grid, stream);
  }
}

}  // namespace asmi
