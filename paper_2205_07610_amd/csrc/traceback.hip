// Traceback: one optimal alignment per pair, in linear memory.
//
// The paper's section 2.1 ("Traceback" paragraph) obtains an alignment by
// following predecessors back through the DP matrices, and its section 3
// notes store predecessors explicitly for short inputs and use Hirschberg's
// divide and conquer for longer ones (linear memory for at most twice the
// cells).  Here, for gfx950:
//
//  - One wave64 per pair (persistent waves take pairs from a counter).
//  - A DP pass is a 64-lane systolic pipeline: lane t owns K = 8 adjacent
//    columns of a 512-column stripe and in step `it` computes row it + 1 - t;
//    H and F of a lane's last column reach lane t + 1 through DPP wave_shr:1,
//    row residues and the left boundary of the stripe are fed to lane 0 in
//    16-row chunks, and lane 63 hands the stripe's right column to the next
//    stripe through a per-wave buffer in global memory (device-coherent
//    loads and stores, so no stale cache line is ever read).  Scores come
//    from an int8 profile of the stripe's columns in LDS.
//  - Affine gaps split the way Myers and Miller extended Hirschberg's
//    method: a subproblem (rows i0..i1, columns j0..j1) is cut at its middle
//    row; a forward pass gives H and E of that row for every column, a pass
//    over the reversed strings gives them for the lower part, and the best
//    column either joins both halves at a cell or joins a vertical gap run
//    that crosses the middle row (then two rows are emitted as gap columns
//    and the halves are told that a run touching that corner continues, so
//    its opening is paid once).  Subproblems go on an explicit stack in LDS,
//    upper part first, so the columns come out in order.
//  - Subproblems of at most 512 columns whose predecessor codes fit 16 KB
//    of LDS (4 bits a cell: the source of H, whether E and F extend) are
//    solved with explicit predecessors and walked back by one lane.
//  - Local and semi-global alignments first find their end cell (forward
//    pass, maximum over all cells / over the last row and column) and their
//    start cell (pass over the reversed prefixes anchored at the end); the
//    optimal alignment is then the global one of that span.
//
// Columns are written as 'M' (q_i against s_j), 'I' (q_i against a gap) and
// 'D' (s_j against a gap), pair p's at ops[(offs_a[p] - offs_a[0]) +
// (offs_b[p] - offs_b[0])]; span[p] = {n_ops, a0, a1, b0, b1}.
#include <mutex>
#include <string.h>
#include <vector>

#include "internal.h"

namespace asmi {
namespace {

constexpr int kTK = 8;                  // columns per lane in a pass
constexpr int kTW = kWave * kTK;        // columns per stripe
constexpr int kTChunk = 16;             // rows per feed refill
constexpr int kTLetters = 32;           // profile rows (largest alphabet)
constexpr int kPredWords = 4096;        // 16 KB of predecessor codes
constexpr int kBaseMaxRows = 512;
constexpr int kTStack = 64;
constexpr unsigned kTbStatusBadOffsets = 1, kTbStatusBadResidue = 2, kTbStatusRange = 4,
                   kTbStatusInternal = 8, kTbStatusStack = 16;

enum TrackMode { kTrackRow = 0, kTrackAll = 1, kTrackEdge = 2, kTrackPred = 3 };

struct TbCounters {
  int32_t next;      // work counter (pairs)
  int32_t status;    // OR of kTbStatus*
  int32_t max_m, max_n;
};

struct TbArgs {
  const uint8_t *seqs_a, *seqs_b;
  const int64_t *offs_a, *offs_b;
  int64_t n_pairs;
  const int8_t *subst;  // device copy, asz * asz
  int asz, alpha, beta, mode;
  int32_t *scores;
  uint8_t *ops;
  int32_t *span;
  TbCounters *ctr;
  int2 *bnd;            // per wave: bnd_stride int2
  int32_t *rows;        // per wave: 4 * row_stride int32 (CC, DD, RR, SS)
  int64_t bnd_stride, row_stride;
  int base_cells;       // explicit predecessors when rows * columns <= this (and they fit LDS)
};

template <int NL>
struct TbShared {
  int8_t prof[NL * kTW];        // NL profile rows (letters) of one stripe's columns
  uint32_t pred[kPredWords + kWave];  // the last kWave words take the stores of lanes past C
  uint8_t opsbuf[kBaseMaxRows + kTW + 8];
  int8_t subst[kTLetters * kTLetters];
  int4 stk[kTStack];
  int stkf[kTStack];
};

__device__ __forceinline__ int t_shr1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xF, 0xF, false);  // wave_shr:1
}
__device__ __forceinline__ int t_shl1(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, 0x130, 0xF, 0xF, false);  // wave_shl:1
}
__device__ __forceinline__ void st_i2(int2 *p, int h, int f) {
  const long long v = (long long)(unsigned)h | ((long long)(unsigned)f << 32);
  __hip_atomic_store((long long *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int2 ld_i2(const int2 *p) {
  const long long v = __hip_atomic_load((const long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_int2((int)(unsigned)(v & 0xffffffffll), (int)(unsigned)((unsigned long long)v >> 32));
}
__device__ __forceinline__ void st_i(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_i(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Score of a horizontal (or a fresh vertical) gap run of k residues.
__device__ __forceinline__ int gap_run(int k, int alpha, int beta) { return k == 0 ? 0 : -alpha - beta * (k - 1); }

struct Best {
  int v, r, c;
};

// Larger value wins; among equal values the smaller (r, c) key.
__device__ __forceinline__ bool better(int v, int key, int bv, int bkey) { return v > bv || (v == bv && key < bkey); }

__device__ Best wave_best(Best b) {
  for (int off = 32; off > 0; off >>= 1) {
    const int ov = __shfl_xor(b.v, off), orr = __shfl_xor(b.r, off), oc = __shfl_xor(b.c, off);
    if (ov > b.v || (ov == b.v && (orr < b.r || (orr == b.r && oc < b.c)))) {
      b.v = ov;
      b.r = orr;
      b.c = oc;
    }
  }
  return b;
}

// One DP pass over the (R + 1) x (C + 1) grid whose row r >= 1 holds residue
// rs[(r - 1) * rdir] and column c >= 1 residue cs[(c - 1) * cdir]
// (R, C >= 1).  Boundary: zero_bnd -- H(r, 0) = H(0, c) = 0 (local,
// semi-global); else H(0, 0) = 0, H(0, c) = -alpha - beta (c - 1),
// H(r, 0) = -open_l - beta (r - 1) (a vertical run from the corner whose
// first residue costs open_l).  E(0, c) = F(r, 0) = -inf; nu is the floor of
// H (0 local, -inf otherwise), Eq. (1),(4),(5).
//   kTrackRow : H and E of row R for columns 0..C into outH / outE (E of
//               column 0 is the boundary run itself)
//   kTrackAll : the largest H over the computed cells
//   kTrackEdge: the largest H over row R and column C, boundary cells
//               (R, 0) and (0, C) included
//   kTrackPred: predecessor codes of every cell into LDS (one stripe), and
//               row R as kTrackRow
template <int TRACK, int NL>
__device__ __noinline__ Best dp_pass(const TbArgs &a, TbShared<NL> &sh, const uint8_t *rs, int rdir, int R, const uint8_t *cs,
                        int cdir, int C, bool zero_bnd, int open_l, int nu, int *outH, int *outE, int2 *bnd) {
  const int t = threadIdx.x;
  const int alpha = a.alpha, beta = a.beta, asz = a.asz;
  const int S = (C + kTW - 1) / kTW;
  const int Pw = (C + kTK - 1) / kTK;  // predecessor words per row (one stripe)
  Best best{kNegInf32, 0x7fffffff, 0x7fffffff};
  auto top = [&](int c) { return (zero_bnd || c == 0) ? 0 : -alpha - beta * (c - 1); };
  auto left = [&](int r) { return (zero_bnd || r == 0) ? 0 : -open_l - beta * (r - 1); };
  if (TRACK == kTrackEdge) {
    // boundary cells (R, 0) and (0, C)
    if (t == 0) {
      const int v0 = left(R), v1 = top(C);
      best = (v1 > v0) ? Best{v1, 0, C} : Best{v0, R, 0};
    }
  }
  if ((TRACK == kTrackRow || TRACK == kTrackPred) && t == 0) {
    st_i(outH, left(R));
    st_i(outE, left(R));  // R >= 1: the boundary column is a vertical run
  }
  for (int s = 0; s < S; ++s) {
    const int c0 = s * kTW + t * kTK;  // this lane's columns c0 + 1 .. c0 + K
    int8_t *pp = sh.prof + t * kTK;
#pragma unroll
    for (int x = 0; x < kTK; ++x) {
      const int c = c0 + x + 1;
      const int code = (c <= C) ? cs[(int64_t)(c - 1) * cdir] : 0;
      for (int l = 0; l < asz; ++l) pp[l * kTW + x] = (c <= C) ? sh.subst[l * asz + code] : (int8_t)0;
    }
    int Hu[kTK], Eu[kTK];
#pragma unroll
    for (int x = 0; x < kTK; ++x) {
      Hu[x] = top(c0 + x + 1);
      Eu[x] = kNegInf32;
    }
    int hl_prev = top(c0);
    int hout = Hu[kTK - 1], fout = kNegInf32;
    int qc = 0;
    const int its = R + kWave - 1;
    const bool import = s > 0, export_ = s + 1 < S;
    int qf = 0, hf = 0, ff = kNegInf32;
    auto load_feed = [&](int it0, int &q, int &h, int &f) {
      if (t < kTChunk) {
        const int r = it0 + t + 1;
        q = 0;
        h = 0;
        f = kNegInf32;
        if (r <= R) {
          q = rs[(int64_t)(r - 1) * rdir];
          if (import) {
            const int2 v = ld_i2(bnd + r);
            h = v.x;
            f = v.y;
          } else {
            h = left(r);
          }
        }
      }
    };
    load_feed(0, qf, hf, ff);
    for (int it0 = 0; it0 < its; it0 += kTChunk) {
      int qn = 0, hn = 0, fn = kNegInf32;
      if (it0 + kTChunk < its) load_feed(it0 + kTChunk, qn, hn, fn);
#pragma unroll 2
      for (int u = 0; u < kTChunk; ++u) {
        const int r = it0 + u + 1 - t;
        qc = t_shr1(qf, qc);
        const int hl = t_shr1(hf, hout);
        const int fl = t_shr1(ff, fout);
        if ((unsigned)(r - 1) < (unsigned)R) {
          const int2 pw = *(const int2 *)(sh.prof + qc * kTW + t * kTK);
          int hleft = hl, fcur = fl, diag = hl_prev;
          uint32_t codes = 0;
#pragma unroll
          for (int x = 0; x < kTK; ++x) {
            const int w32 = (x < 4) ? pw.x : pw.y;
            const int sc = (int)(int8_t)(w32 >> (8 * (x & 3)));
            const int fo = hleft - alpha, fx = fcur - beta;
            const int f = max(fo, fx);
            const int eo = Hu[x] - alpha, ex = Eu[x] - beta;
            const int e = max(eo, ex);
            const int hd = diag + sc;
            int h = max(max(hd, e), f);
            if (nu > kNegInf32) h = max(h, nu);
            if (TRACK == kTrackPred) {
              const uint32_t src = (h == hd) ? 0u : (h == e) ? 1u : 2u;
              codes |= (src | ((ex > eo) ? 4u : 0u) | ((fx > fo) ? 8u : 0u)) << (4 * x);
            }
            if (TRACK == kTrackAll) {
              if (h > best.v) best = {h, r, c0 + x + 1};
            }
            if (TRACK == kTrackEdge) {
              if ((r == R || c0 + x + 1 == C) && c0 + x + 1 <= C && h > best.v) best = {h, r, c0 + x + 1};
            }
            diag = Hu[x];
            Hu[x] = h;
            Eu[x] = e;
            hleft = h;
            fcur = f;
          }
          hout = hleft;
          fout = fcur;
          if (TRACK == kTrackPred) sh.pred[c0 < C ? (r - 1) * Pw + t : kPredWords + t] = codes;
          if ((TRACK == kTrackRow || TRACK == kTrackPred) && r == R) {
#pragma unroll
            for (int x = 0; x < kTK; ++x) {
              const int c = c0 + x + 1;
              if (c <= C) {
                st_i(outH + c, Hu[x]);
                st_i(outE + c, Eu[x]);
              }
            }
          }
          if (export_ && t == kWave - 1) st_i2(bnd + r, hout, fout);
        }
        hl_prev = hl;
        qf = t_shl1(qf, qf);
        hf = t_shl1(hf, hf);
        ff = t_shl1(ff, ff);
      }
      qf = qn;
      hf = hn;
      ff = fn;
    }
    // the next stripe reads this stripe's right column: wait for the stores
    __threadfence();
  }
  if (TRACK == kTrackAll || TRACK == kTrackEdge) best = wave_best(best);
  __threadfence();
  __syncthreads();
  return best;
}

// Emit `k` copies of op at ops[cur..cur + k) (the whole wave writes).
__device__ __forceinline__ void emit_run(uint8_t *ops, int64_t cur, int k, uint8_t op) {
  for (int i = threadIdx.x; i < k; i += kWave) ops[cur + i] = op;
}

// Explicit-predecessor base case of subproblem rows [i0, i1) x columns
// [j0, j1) (1 <= C <= one stripe, predecessor codes fit LDS), vertical runs
// touching the top-left corner continue from above when ct, runs touching the
// bottom-right corner continue below when cb.  Returns the value; the
// alignment's columns go to ops[cur ..], their number to *n_out.
template <int NL>
__device__ __noinline__ int base_case(const TbArgs &a, TbShared<NL> &sh, const uint8_t *A, const uint8_t *B, int i0, int i1, int j0,
                         int j1, int ct, int cb, uint8_t *ops, int64_t cur, int *n_out, int *rowsH, int *rowsE) {
  const int R = i1 - i0, C = j1 - j0;
  const int alpha = a.alpha, beta = a.beta;
  dp_pass<kTrackPred, NL>(a, sh, A + i0, 1, R, B + j0, 1, C, false, ct ? beta : alpha, kNegInf32, rowsH, rowsE,
                      nullptr);
  const int Pw = (C + kTK - 1) / kTK;
  int value = 0, len = 0;
  if (threadIdx.x == 0) {
    const int hR = ld_i(rowsH + C), eR = ld_i(rowsE + C);
    int state = 0;  // 0: H, 1: E (vertical run), 2: F (horizontal run)
    value = hR;
    if (cb && eR + (alpha - beta) > hR) {
      value = eR + (alpha - beta);
      state = 1;
    }
    int r = R, c = C;
    uint8_t *buf = sh.opsbuf;
    for (;;) {
      if (r == 0) {
        for (; c > 0; --c) buf[len++] = 'D';
        break;
      }
      if (c == 0) {
        for (; r > 0; --r) buf[len++] = 'I';
        break;
      }
      const uint32_t code = (sh.pred[(r - 1) * Pw + (c - 1) / kTK] >> (4 * ((c - 1) % kTK))) & 15u;
      if (state == 0) {
        const uint32_t src = code & 3u;
        if (src == 0) {
          buf[len++] = 'M';
          --r;
          --c;
        } else {
          state = (src == 1) ? 1 : 2;
        }
      } else if (state == 1) {
        buf[len++] = 'I';
        state = (code & 4u) ? 1 : 0;
        --r;
      } else {
        buf[len++] = 'D';
        state = (code & 8u) ? 2 : 0;
        --c;
      }
    }
  }
  __syncthreads();
  len = __shfl(len, 0);
  value = __shfl(value, 0);
  for (int k = threadIdx.x; k < len; k += kWave) ops[cur + k] = sh.opsbuf[len - 1 - k];
  __syncthreads();
  *n_out = len;
  return value;
}

// One row (R == 1) against C columns: the residue aligned to one column with
// gap runs around it, or deleted before or after a run over every column.
template <int NL>
__device__ __noinline__ int one_row(const TbArgs &a, TbShared<NL> &sh, const uint8_t *A, const uint8_t *B, int i0, int j0, int C,
                       int ct, int cb, uint8_t *ops, int64_t cur, int *n_out) {
  const int alpha = a.alpha, beta = a.beta;
  const int q = A[i0];
  Best b{kNegInf32, 0, 0x7fffffff};
  for (int j = threadIdx.x + 1; j <= C; j += kWave) {
    const int v = gap_run(j - 1, alpha, beta) + sh.subst[q * a.asz + B[j0 + j - 1]] + gap_run(C - j, alpha, beta);
    if (v > b.v) b = {v, 0, j};
  }
  b = wave_best(b);
  const int first = -(ct ? beta : alpha) + gap_run(C, alpha, beta);
  const int last = gap_run(C, alpha, beta) - (cb ? beta : alpha);
  int value = b.v, kind = 0;
  if (first > value) { value = first; kind = 1; }
  if (last > value) { value = last; kind = 2; }
  if (kind == 0) {
    const int j = b.c;
    emit_run(ops, cur, j - 1, 'D');
    if (threadIdx.x == 0) ops[cur + j - 1] = 'M';
    emit_run(ops, cur + j, C - j, 'D');
  } else if (kind == 1) {
    if (threadIdx.x == 0) ops[cur] = 'I';
    emit_run(ops, cur + 1, C, 'D');
  } else {
    emit_run(ops, cur, C, 'D');
    if (threadIdx.x == 0) ops[cur + C] = 'I';
  }
  *n_out = (kind == 0) ? C : C + 1;
  return value;
}

// Global alignment of A[i0..i1) against B[j0..j1) by divide and conquer;
// returns the optimal value, writes the columns from ops[cur] on and returns
// their number in *n_ops.
template <int NL>
__device__ int solve(const TbArgs &a, TbShared<NL> &sh, const uint8_t *A, const uint8_t *B, int i0, int i1, int j0,
                     int j1, uint8_t *ops, int64_t cur0, int *n_ops, int2 *bnd, int *rows) {
  const int t = threadIdx.x;
  const int alpha = a.alpha, beta = a.beta;
  const int64_t rs = a.row_stride;
  int *CC = rows, *DD = rows + rs, *RR = rows + 2 * rs, *SS = rows + 3 * rs;
  int sp = 0;
  if (t == 0) {
    sh.stk[0] = make_int4(i0, i1, j0, j1);
    sh.stkf[0] = 0;
  }
  sp = 1;
  __syncthreads();
  int64_t cur = cur0;
  int root_value = 0;
  bool first = true;
  while (sp > 0) {
    --sp;
    const int4 tk = sh.stk[sp];
    const int fl = sh.stkf[sp];
    __syncthreads();
    const int ct = fl & 1, cb = (fl >> 1) & 1;
    const int R = tk.y - tk.x, C = tk.w - tk.z;
    int value = 0, n = 0;
    if (fl & 4) {  // two vertical gap columns of a run crossing a middle row
      if (t == 0) {
        ops[cur] = 'I';
        ops[cur + 1] = 'I';
      }
      cur += 2;
      continue;
    }
    if (R == 0) {
      emit_run(ops, cur, C, 'D');
      value = gap_run(C, alpha, beta);
      n = C;
    } else if (C == 0) {
      emit_run(ops, cur, R, 'I');
      value = (ct || cb) ? -beta * R : gap_run(R, alpha, beta);
      n = R;
    } else if (C <= kTW && R <= kBaseMaxRows && R * ((C + kTK - 1) / kTK) <= kPredWords &&
               (int64_t)R * C <= a.base_cells) {
      value = base_case(a, sh, A, B, tk.x, tk.y, tk.z, tk.w, ct, cb, ops, cur, &n, CC, DD);
    } else if (R == 1) {
      value = one_row(a, sh, A, B, tk.x, tk.z, C, ct, cb, ops, cur, &n);
    } else {
      const int mid = tk.x + R / 2;
      const int Ru = mid - tk.x, Rl = tk.y - mid;
      dp_pass<kTrackRow, NL>(a, sh, A + tk.x, 1, Ru, B + tk.z, 1, C, false, ct ? beta : alpha, kNegInf32, CC, DD,
                         bnd);
      dp_pass<kTrackRow, NL>(a, sh, A + tk.y - 1, -1, Rl, B + tk.w - 1, -1, C, false, cb ? beta : alpha, kNegInf32,
                         RR, SS, bnd);
      // best column: a cell of the middle row (type 1) or a vertical run
      // through it (type 2); ties to the smaller column, then type 1
      int bv = kNegInf32 * 2, bkey = 0x7fffffff;
      for (int j = t; j <= C; j += kWave) {
        const int v1 = ld_i(CC + j) + ld_i(RR + (C - j));
        const int v2 = ld_i(DD + j) + ld_i(SS + (C - j)) + (alpha - beta);
        if (better(v1, 2 * j, bv, bkey)) { bv = v1; bkey = 2 * j; }
        if (better(v2, 2 * j + 1, bv, bkey)) { bv = v2; bkey = 2 * j + 1; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const int ov = __shfl_xor(bv, off), ok = __shfl_xor(bkey, off);
        if (better(ov, ok, bv, bkey)) { bv = ov; bkey = ok; }
      }
      value = bv;
      const int j = tk.z + (bkey >> 1);
      if (sp + 3 > kTStack) {
        if (t == 0) atomicOr(&a.ctr->status, kTbStatusStack);
        *n_ops = 0;
        return value;
      }
      if (t == 0) {
        if ((bkey & 1) == 0) {
          sh.stk[sp] = make_int4(mid, tk.y, j, tk.w);
          sh.stkf[sp] = (cb << 1);
          sh.stk[sp + 1] = make_int4(tk.x, mid, tk.z, j);
          sh.stkf[sp + 1] = ct;
        } else {
          sh.stk[sp] = make_int4(mid + 1, tk.y, j, tk.w);
          sh.stkf[sp] = 1 | (cb << 1);
          sh.stk[sp + 1] = make_int4(0, 0, 0, 0);
          sh.stkf[sp + 1] = 4;
          sh.stk[sp + 2] = make_int4(tk.x, mid - 1, tk.z, j);
          sh.stkf[sp + 2] = ct | 2;
        }
      }
      sp += ((bkey & 1) == 0) ? 2 : 3;
      __syncthreads();
      if (first) root_value = value;
      first = false;
      continue;
    }
    if (first) root_value = value;
    first = false;
    cur += n;
  }
  *n_ops = (int)(cur - cur0);
  return root_value;
}

template <int NL>
__global__ void __launch_bounds__(kWave) traceback_kernel(TbArgs a) {
  __shared__ __align__(16) TbShared<NL> sh;
  const int t = threadIdx.x;
  for (int i = t; i < a.asz * a.asz; i += kWave) sh.subst[i] = a.subst[i];
  __syncthreads();
  int2 *bnd = a.bnd + (int64_t)blockIdx.x * a.bnd_stride;
  int *rows = a.rows + (int64_t)blockIdx.x * 4 * a.row_stride;
  const int64_t oa0 = a.offs_a[0], ob0 = a.offs_b[0];
  const int alpha = a.alpha;
  for (;;) {
    int p = 0;
    if (t == 0) p = atomicAdd(&a.ctr->next, 1);
    p = __shfl(p, 0);
    if (p >= a.n_pairs) break;
    const int64_t ao = a.offs_a[p], bo = a.offs_b[p];
    const int m = (int)(a.offs_a[p + 1] - ao), n = (int)(a.offs_b[p + 1] - bo);
    const uint8_t *A = a.seqs_a + ao, *B = a.seqs_b + bo;
    uint8_t *ops = a.ops + (ao - oa0) + (bo - ob0);
    int a0 = 0, a1 = m, b0 = 0, b1 = n, score = 0, nops = 0;
    bool run = true;
    if (a.mode == kGlobal) {
      // the whole matrix
    } else if (m == 0 || n == 0) {
      a0 = a1 = b0 = b1 = 0;  // the empty alignment scores 0 (nothing better exists)
      run = false;
    } else if (a.mode == kLocal) {
      const Best e = dp_pass<kTrackAll, NL>(a, sh, A, 1, m, B, 1, n, true, 0, 0, nullptr, nullptr, bnd);
      if (e.v <= 0) {
        a0 = a1 = b0 = b1 = 0;
        run = false;
      } else {
        a1 = e.r;
        b1 = e.c;
        const Best st = dp_pass<kTrackAll, NL>(a, sh, A + a1 - 1, -1, a1, B + b1 - 1, -1, b1, false, alpha, kNegInf32,
                                           nullptr, nullptr, bnd);
        a0 = a1 - st.r;
        b0 = b1 - st.c;
        score = e.v;
        if (st.v != e.v && t == 0) atomicOr(&a.ctr->status, kTbStatusInternal);
      }
    } else {
      const Best e = dp_pass<kTrackEdge, NL>(a, sh, A, 1, m, B, 1, n, true, 0, kNegInf32, nullptr, nullptr, bnd);
      a1 = e.r;
      b1 = e.c;
      score = e.v;
      if (a1 == 0 || b1 == 0) {
        a0 = a1;
        b0 = b1;
        run = false;
      } else {
        const Best st = dp_pass<kTrackEdge, NL>(a, sh, A + a1 - 1, -1, a1, B + b1 - 1, -1, b1, false, alpha,
                                            kNegInf32, nullptr, nullptr, bnd);
        a0 = a1 - st.r;
        b0 = b1 - st.c;
        if (st.v != e.v && t == 0) atomicOr(&a.ctr->status, kTbStatusInternal);
      }
    }
    if (run) {
      const int v = solve(a, sh, A, B, a0, a1, b0, b1, ops, 0, &nops, bnd, rows);
      if (a.mode == kGlobal) score = v;
      else if (v != score && t == 0) atomicOr(&a.ctr->status, kTbStatusInternal);
    }
    if (t == 0) {
      a.scores[p] = score;
      int32_t *sp = a.span + 5 * p;
      sp[0] = nops;
      sp[1] = a0;
      sp[2] = a1;
      sp[3] = b0;
      sp[4] = b1;
    }
    __syncthreads();
  }
}

// Offsets, residues and the 32-bit range of every pair; the longest row and
// column sequences (they size the per-wave buffers).
__global__ void __launch_bounds__(256) traceback_prep_kernel(TbArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t budget = (int64_t)1 << 28;
  int smax = 0;
  for (int i = 0; i < a.asz * a.asz; ++i) smax = max(smax, abs((int)a.subst[i]));
  int mm = 0, mn = 0;
  for (int64_t p = g; p < a.n_pairs; p += stride) {
    const int64_t a0 = a.offs_a[p], a1 = a.offs_a[p + 1], b0 = a.offs_b[p], b1 = a.offs_b[p + 1];
    if (a0 < 0 || b0 < 0 || a1 < a0 || b1 < b0 || a0 < a.offs_a[0] || b0 < a.offs_b[0]) {
      atomicOr(&a.ctr->status, kTbStatusBadOffsets);
      continue;
    }
    const int64_t m = a1 - a0, n = b1 - b0;
    if (m >= ((int64_t)1 << 30) || n >= ((int64_t)1 << 30) ||
        (int64_t)(smax + a.alpha + 2 * a.beta) * (m + n + 2) >= budget) {
      atomicOr(&a.ctr->status, kTbStatusRange);
      continue;
    }
    mm = max(mm, (int)m);
    mn = max(mn, (int)n);
  }
  atomicMax(&a.ctr->max_m, mm);
  atomicMax(&a.ctr->max_n, mn);
}

__global__ void __launch_bounds__(256) traceback_residue_kernel(const uint8_t *s, int64_t lo, int64_t hi, int asz,
                                                                int32_t *status) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride)
    bad |= s[i] >= asz;
  if (bad) atomicOr(status, kTbStatusBadResidue);
}

struct TbWork {
  int device = -1;
  int num_cu = 0;
  TbCounters *ctr = nullptr;
  TbCounters *host = nullptr;  // pinned
  int8_t *subst = nullptr;
  void *scratch = nullptr;
  int64_t scratch_bytes = 0;
};

std::mutex g_tlock;
std::vector<TbWork> g_tw;
int g_base_cells = 1 << 30;

#define TB_HIP(call)                             \
  do {                                           \
    if ((call) != hipSuccess) return AS_ERR_HIP; \
  } while (0)

int tb_work(TbWork **out) {
  int dev = 0;
  TB_HIP(hipGetDevice(&dev));
  if ((int)g_tw.size() <= dev) g_tw.resize(dev + 1);
  TbWork &w = g_tw[dev];
  if (w.device < 0) {
    hipDeviceProp_t prop;
    TB_HIP(hipGetDeviceProperties(&prop, dev));
    w.num_cu = prop.multiProcessorCount;
    TB_HIP(hipMalloc(&w.ctr, sizeof(TbCounters)));
    TB_HIP(hipHostMalloc(&w.host, sizeof(TbCounters), hipHostMallocDefault));
    TB_HIP(hipMalloc(&w.subst, kTLetters * kTLetters));
    w.device = dev;
  }
  *out = &w;
  return AS_OK;
}

int tb_status_code(int32_t st) {
  if (st & kTbStatusBadOffsets) return AS_ERR_OFFSETS;
  if (st & kTbStatusBadResidue) return AS_ERR_RESIDUE;
  if (st & kTbStatusRange) return AS_ERR_RANGE;
  if (st & (kTbStatusInternal | kTbStatusStack)) return AS_ERR_HIP;
  return AS_OK;
}

}  // namespace

void release_traceback_workspace() {
  std::lock_guard<std::mutex> guard(g_tlock);
  for (TbWork &w : g_tw) {
    if (w.device < 0) continue;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(w.device);
    if (w.ctr) (void)hipFree(w.ctr);
    if (w.host) (void)hipHostFree(w.host);
    if (w.subst) (void)hipFree(w.subst);
    if (w.scratch) (void)hipFree(w.scratch);
    (void)hipSetDevice(cur);
    w = TbWork();
  }
}

}  // namespace asmi

using namespace asmi;

extern "C" int as_align_batch_traceback(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                                        const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                                        int32_t mode, int32_t *scores_out, uint8_t *ops_out, int32_t *span_out,
                                        void *stream_ptr) {
  if (!scoring || !scoring->subst || !seqs_a || !seqs_b || !offs_a || !offs_b || !scores_out || !ops_out ||
      !span_out)
    return AS_ERR_NULL;
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31) - 1) return AS_ERR_ARG;
  const int asz = scoring->alphabet_size, alpha = scoring->gap_open, beta = scoring->gap_extend;
  if (asz < 2 || asz > kTLetters || beta < 0 || alpha < beta || alpha > 10000 || mode < 0 || mode > 2)
    return AS_ERR_SCORING;
  if (n_pairs == 0) return AS_OK;
  std::lock_guard<std::mutex> guard(g_tlock);
  TbWork *w = nullptr;
  int rc = tb_work(&w);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_ptr;
  TbArgs a;
  memset(&a, 0, sizeof(a));
  a.seqs_a = seqs_a;
  a.seqs_b = seqs_b;
  a.offs_a = offs_a;
  a.offs_b = offs_b;
  a.n_pairs = n_pairs;
  a.subst = w->subst;
  a.asz = asz;
  a.alpha = alpha;
  a.beta = beta;
  a.mode = mode;
  a.scores = scores_out;
  a.ops = ops_out;
  a.span = span_out;
  a.ctr = w->ctr;
  a.base_cells = g_base_cells;
  TB_HIP(hipMemcpyAsync(w->subst, scoring->subst, (size_t)asz * asz, hipMemcpyHostToDevice, stream));
  TB_HIP(hipMemsetAsync(w->ctr, 0, sizeof(TbCounters), stream));
  int64_t blocks = (n_pairs + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(traceback_prep_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  TB_HIP(hipGetLastError());
  TB_HIP(hipMemcpyAsync(w->host, w->ctr, sizeof(TbCounters), hipMemcpyDeviceToHost, stream));
  TB_HIP(hipStreamSynchronize(stream));
  TbCounters c = *w->host;
  if ((rc = tb_status_code(c.status))) return rc;
  // residues of the whole batch (the offsets are valid now)
  int64_t ends[4];
  TB_HIP(hipMemcpyAsync(&ends[0], offs_a, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
  TB_HIP(hipMemcpyAsync(&ends[1], offs_a + n_pairs, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
  TB_HIP(hipMemcpyAsync(&ends[2], offs_b, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
  TB_HIP(hipMemcpyAsync(&ends[3], offs_b + n_pairs, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
  TB_HIP(hipStreamSynchronize(stream));
  hipLaunchKernelGGL(traceback_residue_kernel, dim3(1024), dim3(256), 0, stream, seqs_a, ends[0], ends[1], asz,
                     &w->ctr->status);
  TB_HIP(hipGetLastError());
  hipLaunchKernelGGL(traceback_residue_kernel, dim3(1024), dim3(256), 0, stream, seqs_b, ends[2], ends[3], asz,
                     &w->ctr->status);
  TB_HIP(hipGetLastError());
  TB_HIP(hipMemcpyAsync(w->host, w->ctr, sizeof(TbCounters), hipMemcpyDeviceToHost, stream));
  TB_HIP(hipStreamSynchronize(stream));
  c = *w->host;
  if ((rc = tb_status_code(c.status))) return rc;
  // persistent waves; per wave the stripe boundary column (rows + 2) and the
  // four middle-row vectors (columns + 2)
  int per_cu = 0;
  const bool small_alphabet = asz <= 4;
  const hipError_t oe = small_alphabet
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, traceback_kernel<4>, kWave, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, traceback_kernel<kTLetters>, kWave, 0);
  if (oe != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)per_cu * w->num_cu;
  if (grid > n_pairs) grid = n_pairs;
  a.bnd_stride = ((int64_t)c.max_m + 2 + 31) & ~(int64_t)31;
  a.row_stride = ((int64_t)c.max_n + 2 + 63) & ~(int64_t)63;
  const int64_t need = grid * (a.bnd_stride * (int64_t)sizeof(int2) + 4 * a.row_stride * (int64_t)sizeof(int32_t));
  if (w->scratch_bytes < need) {
    if (w->scratch) (void)hipFree(w->scratch);
    w->scratch = nullptr;
    w->scratch_bytes = 0;
    TB_HIP(hipMalloc(&w->scratch, (size_t)need));
    w->scratch_bytes = need;
  }
  a.bnd = (int2 *)w->scratch;
  a.rows = (int32_t *)((char *)w->scratch + grid * a.bnd_stride * (int64_t)sizeof(int2));
  if (small_alphabet)
    hipLaunchKernelGGL(traceback_kernel<4>, dim3((unsigned)grid), dim3(kWave), 0, stream, a);
  else
    hipLaunchKernelGGL(traceback_kernel<kTLetters>, dim3((unsigned)grid), dim3(kWave), 0, stream, a);
  TB_HIP(hipGetLastError());
  TB_HIP(hipMemcpyAsync(w->host, w->ctr, sizeof(TbCounters), hipMemcpyDeviceToHost, stream));
  TB_HIP(hipStreamSynchronize(stream));
  return tb_status_code(w->host->status);
}

extern "C" int as_set_traceback_base(int32_t cells) {
  std::lock_guard<std::mutex> guard(g_tlock);
  const int prev = g_base_cells;
  g_base_cells = cells <= 0 ? (1 << 30) : cells;
  return prev;
}
