/*
 * anyseq_mi -- score-only pairwise alignment of large batches of sequence
 * pairs on AMD Instinct MI355X (gfx950).
 *
 * The problem follows the statement of AnySeq/GPU (arXiv 2205.07610),
 * section 2.1: pairs (Q, S) of sequences over an alphabet, a substitution
 * function sigma over alphabet x alphabet, gap penalties alpha (first gap
 * residue) and beta (each further residue), so a gap of length k costs
 * alpha + (k-1)*beta (Eq. (4),(5); linear gaps are alpha == beta, Eq. (2),(3)),
 * and an alignment type: global, semi-global or local (the mode paragraphs
 * of section 2.1).  Batches of pairs go in, one optimal score per pair comes
 * out (the paper's Listing 1 signature; score-only, "Traceback" paragraph).
 *
 * Conventions shared by every entry point
 *  - Sequences are residue codes 0..alphabet_size-1, one byte per residue,
 *    concatenated: pair p is A[offs_a[p] .. offs_a[p+1]) against
 *    B[offs_b[p] .. offs_b[p+1]).  Offsets are int64, non-decreasing,
 *    offs[0] >= 0; the caller guarantees the sequence buffers hold
 *    offs[n_pairs] bytes.  Empty sequences are allowed.
 *  - Rows of the dynamic program run over A (q_i, i = 1..m), columns over
 *    B (s_j, j = 1..n), sigma(q_i, s_j) = subst[q_i * alphabet_size + s_j].
 *    The library may transpose a pair internally; results are unchanged.
 *  - Device pointers are HIP device memory on the current device; the caller
 *    owns every buffer.  `stream` is a hipStream_t (NULL = default stream).
 *    Calls are stream-ordered; the return code is known when the call
 *    returns (the call waits for its own status word).
 *  - Errors: a negative return code; scores_out contents are then
 *    unspecified.  A call never returns 0 with a wrong score.  No C++
 *    exception crosses this interface.
 *  - Scratch memory is owned by the library, cached per device and grown on
 *    demand; as_release_workspace() frees it.  Calls on one device are
 *    serialised by the library (a process-wide lock).
 */
#ifndef ANYSEQ_MI_H
#define ANYSEQ_MI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Alignment type (paper section 2.1). */
typedef enum {
    AS_GLOBAL = 0,     /* nu = -inf, penalised end gaps, result H(m,n) */
    AS_SEMIGLOBAL = 1, /* free end gaps: result = max over last row and column */
    AS_LOCAL = 2       /* Smith-Waterman: nu = 0, result = max over all cells */
} as_mode;

/* Scoring scheme.  All penalties are magnitudes that are subtracted. */
typedef struct {
    int32_t alphabet_size; /* 2..32 */
    const int8_t *subst;   /* HOST pointer, alphabet_size^2 entries, row-major */
    int32_t gap_open;      /* alpha: cost of a gap's first residue */
    int32_t gap_extend;    /* beta: cost of each further residue, 0 <= beta <= alpha */
} as_scoring;
/*
 * Limits of a scoring scheme (AS_ERR_SCORING otherwise): with bias =
 * alpha + beta (global, semi-global) or alpha (local), bias <= 127 and every
 * sigma + bias lies in -128..127 (the 32-bit kernels keep sigma + bias as one
 * signed byte per letter and column).  The banded and learned entry points
 * also need at most four letters and sigma + alpha + beta in 0..255.
 */

/* Return codes. */
#define AS_OK 0
#define AS_ERR_NULL (-1)      /* a required pointer is NULL */
#define AS_ERR_OFFSETS (-2)   /* offsets decrease or offs[0] < 0 */
#define AS_ERR_RESIDUE (-3)   /* a residue code >= alphabet_size */
#define AS_ERR_SCORING (-4)   /* alphabet size, alpha, beta or mode invalid */
#define AS_ERR_RANGE (-5)     /* a score could leave the int32 range */
#define AS_ERR_HIP (-6)       /* a HIP runtime call failed, or a device-side wait stalled */
#define AS_ERR_ARG (-7)       /* another argument is out of range */
#define AS_ERR_SCRATCH (-8)   /* as_align_batch_noalloc: the batch does not fit its scratch array */

/*
 * Optimal alignment score of every pair of the batch (paper section 2.1,
 * Eq. (1),(4),(5), mode as given).
 *   seqs_a, seqs_b : device, uint8 residue codes
 *   offs_a, offs_b : device, int64 [n_pairs + 1]
 *   n_pairs        : >= 0 (0 returns AS_OK and touches nothing)
 *   scoring        : host struct, read during the call only
 *   mode           : as_mode
 *   scores_out     : device, int32 [n_pairs]
 *   stream         : hipStream_t or NULL
 * Pairs whose scores fit 16-bit cells (a priori bound, or no saturation at
 * run time) take the packed 16-bit path; all others, and every 16-bit pair
 * that saturates, are computed with 32-bit cells.  Results are exact in
 * every case.
 */
int as_align_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                   const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                   int32_t mode, int32_t *scores_out, void *stream);

/*
 * All against all (the paper's evaluation workload, section 4.1: every read
 * of a set aligned with every read of a set): the score of query q against
 * subject s for every q < n_q and s < n_s, Eq. (1),(4),(5) in the given mode.
 *   seqs_q, offs_q : device, the n_q query sequences (offs_q[n_q + 1])
 *   seqs_s, offs_s : device, the n_s subject sequences (offs_s[n_s + 1])
 *   scores_out     : device int32 [n_q][n_s], row-major (query q, subject s
 *                    at scores_out[q * n_s + s])
 * Rows of each DP are the query's residues, columns the subject's; sigma
 * is indexed (query letter, subject letter).  n_q * n_s must stay below
 * 2^31 - 1 (AS_ERR_ARG).  Offsets of the two sets are copied to the host to
 * validate them and find the longest sequences (AS_ERR_OFFSETS,
 * AS_ERR_RANGE for the longest query against the longest subject).  When
 * one set's sequences fit one packed stripe (at most 256 residues), the
 * alphabet has at most 4 letters and (global, semi-global) the longest pair
 * passes the packed range proof, one kernel computes every pair with the
 * pairs implicit: a wave builds the register profile of one sequence of
 * that set once and keeps it for a block of sequences of the other set
 * (the paper's section 3.1 profile, built once per subject and reused).
 * Other batches go through as_align_batch's routing and kernels in chunks.
 * Same errors as as_align_batch.
 */
int as_align_all_vs_all(const uint8_t *seqs_q, const int64_t *offs_q, int64_t n_q,
                        const uint8_t *seqs_s, const int64_t *offs_s, int64_t n_s,
                        const as_scoring *scoring, int32_t mode, int32_t *scores_out, void *stream);

/*
 * as_align_batch for callers that cannot allocate memory (code that runs
 * while a HIP graph is being captured elsewhere, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, same results, same
 * kernels, but the call allocates nothing -- no hipMalloc/hipFree, no
 * pinned host buffer, no library routine that allocates.  Its work lists,
 * counters and boundary buffers live in one static device array of
 * AS_NOALLOC_SCRATCH_BYTES per GPU, held by the process until it ends.
 * Limits: the five work lists take 176 bytes per pair and the long-pair
 * boundary columns 8 bytes per row per stripe edge, all within that array
 * (about 380,000 short pairs; a batch whose long pairs need more boundary
 * rows than remain is refused); a batch that does not fit returns
 * AS_ERR_SCRATCH before its DP kernels run.  The first call on a device
 * looks up the array's device address (hipGetSymbolAddress).  Every call on
 * a GPU shares that GPU's array and leaves its contents behind; the call
 * clears what must start at zero.  Calls from one process are serialised
 * by the library's lock and wait for their own work before returning, so
 * they never overlap; calls that overlapped on one GPU (for example from
 * two copies of the library in one process) would race on the array.
 * Timing (as_enable_timing) is not recorded for these calls.
 */
#define AS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int as_align_batch_noalloc(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                           const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                           int32_t mode, int32_t *scores_out, void *stream);

/*
 * One optimal alignment of every pair, besides its score (paper section 2.1,
 * "Traceback" paragraph: the alignment is found by following predecessors
 * back; section 3's implementation notes: explicit predecessors for short
 * inputs, Hirschberg's linear-space divide and conquer for longer ones).
 * Arguments as as_align_batch, plus
 *   ops_out  : device, uint8, at least (offs_a[n] - offs_a[0]) +
 *              (offs_b[n] - offs_b[0]) bytes (>= 1).  Pair p's alignment
 *              columns start at ops_out[(offs_a[p] - offs_a[0]) +
 *              (offs_b[p] - offs_b[0])] and take at most m + n bytes: 'M'
 *              aligns q_i with s_j (match or mismatch), 'I' puts q_i against
 *              a gap, 'D' puts s_j against a gap, first column first.
 *   span_out : device, int32 [n_pairs][5] = {n_ops, a0, a1, b0, b1}: the
 *              alignment covers A[a0..a1) and B[b0..b1).  Global: the whole
 *              of both sequences.  Semi-global: a0 == 0 or b0 == 0, and
 *              a1 == m or b1 == n (the cut-off ends are the free end gaps).
 *              Local: any substrings; score 0 gives the empty alignment.
 * The alignment's score by the definition (sigma over 'M' columns,
 * alpha + (k-1) beta per maximal run of k equal gap columns) equals
 * scores_out[p], the optimal score.  When several alignments are optimal,
 * which one is returned is unspecified.  Cells are 32-bit; the same range
 * limit as as_align_batch applies (AS_ERR_RANGE).  Work: at most about four
 * times the pair's cells for local and semi-global pairs (end cell, start
 * cell, twice the span's cells), twice for global ones; memory: the library
 * keeps per resident wave a column of (longest A + 2) and four rows of
 * (longest B + 2) 32-bit values.
 */
int as_align_batch_traceback(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                             const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                             int32_t mode, int32_t *scores_out, uint8_t *ops_out, int32_t *span_out,
                             void *stream);

/*
 * Test hook of the traceback: subproblems of at most `cells` cells (and
 * within the kernel's LDS limits) are solved with explicit predecessors,
 * larger ones are split; <= 0 restores the default (as large as LDS
 * allows).  Returns the previous value.
 */
int as_set_traceback_base(int32_t cells);

/* Human-readable text for a return code (static storage). */
const char *as_strerror(int code);

/* Free the library's cached scratch memory on every device.  Returns AS_OK. */
int as_release_workspace(void);

/* Build information: the offload target and the kernel variants compiled in. */
const char *as_build_info(void);

/*
 * Per-phase GPU times of the most recent as_align_batch call on this
 * process, measured with HIP events recorded on the call's stream around
 * each phase (only while timing is enabled; disabled by default because the
 * events cost a few microseconds per call).  Times are milliseconds; a phase
 * that did not run reports 0.  Counts describe the same call.
 */
typedef struct {
    float classify_ms;  /* validation, orientation, work lists */
    float full32_ms;    /* full DP, 32-bit cells */
    float full16_ms;    /* full DP, packed 16-bit cells */
    float rerun32_ms;   /* 32-bit re-run of saturated 16-bit pairs */
    float long_ms;      /* multi-wave wavefront for long pairs, 32-bit cells */
    float band_ms;      /* banded rounds (as_align_batch_band) */
    float features_ms;  /* k-mer features (as_align_batch_learned) */
    float mlp_ms;       /* band network inference (as_align_batch_learned) */
    float band16_ms;    /* part of band_ms spent in the packed 16-bit banded kernel */
    float long16_ms;    /* packed 16-bit wavefront for long global pairs, two per wave */
    int64_t pairs_full32;
    int64_t pairs_full16;
    int64_t pairs_rerun32;
    int64_t pairs_long;
    int64_t pairs_fallback; /* banded pairs that went to the full DP */
    int64_t cells;      /* sum of m*n over the batch */
    int64_t cells_full32;   /* sum of m*n of the pairs of each full-DP route */
    int64_t cells_full16;
    int64_t cells_long;
    int64_t pairs_long16;
    int64_t cells_long16;
    int64_t full16_cell_type; /* cells of the packed full-DP kernel: 0 int16, 1 FP16 with FP8 E4M3
                                 profile bytes, 2 FP16 with FP8 E5M2 profile bytes */
    int64_t full32_variants;  /* variants the 32-bit list ran: bit 0 K = 8, bit 1 K = 16, bit 2 K = 32,
                                 bit 3 the packed int16 LDS-profile variant (two local pairs per group) */
} as_timing;

/*
 * Banded path with a certificate (the learned-band extension; not in the
 * paper).  For global and semi-global alignment of alphabets of at most four
 * letters.  Pair p is first aligned inside the band of diagonals
 *   min(0, n-m) - w <= j - i <= max(0, n-m) + w,   w = band_w0[p]
 * widened to the kernel's lane width (a band of 64..1536 diagonals,
 * centred on the requested one).  The banded score is accepted when it is at
 * least an upper bound on every alignment path that leaves the computed band
 * (closed form from the path structure of Eq. (1),(4),(5)); then it is the
 * optimal score.  Otherwise, for at most max_rounds rounds (1..8), the next
 * half-width is (global) the smallest one whose bound the rejected score
 * would pass, or (semi-global) twice w.  A band is used only when some lane
 * width holds it: at most 1536 diagonals, and less than half the longer sequence (32-bit cells) or at
 * most three quarters of it (packed 16-bit cells, global mode).  A request
 * that no width holds -- the initial one, or a widened one when a wider band
 * than the last round's exists and the rejected score does not already rule
 * it out -- takes the widest band the pair allows instead.  A pair with no band left, or out of rounds, is aligned with the
 * full DP.  Every returned score is exact.
 *   band_w0    : device, int32 [n_pairs], initial half-widths (< 0 read as 0)
 *   stats      : HOST, optional (NULL), filled on return
 * Local mode returns AS_ERR_ARG; alphabets above four letters, or scores
 * sigma + alpha + beta outside 0..255, return AS_ERR_SCORING.
 */
typedef struct {
    int32_t rounds;        /* banded rounds that ran */
    int32_t reserved;
    int64_t accepted[8];   /* pairs accepted in round r */
    int64_t fallback;      /* pairs aligned with the full DP */
    int64_t band_cells;    /* DP cells computed by the banded kernel */
    int64_t cells;         /* sum of m*n over the batch */
    int64_t fallback_cells; /* sum of m*n over the pairs aligned with the full DP */
    int64_t band16_cells;  /* part of band_cells computed with packed 16-bit cells */
} as_band_stats;

int as_align_batch_band(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                        const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                        int32_t mode, const int32_t *band_w0, int32_t max_rounds,
                        int32_t *scores_out, as_band_stats *stats, void *stream);

/*
 * Raw banded scores: the optimal score of pair p restricted to the band the
 * kernel computes for half-width band_w[p] (see above), with no acceptance
 * test.  The kernel is the one the certified rounds would use: in global
 * mode the packed 16-bit kernel (widths 80..1536) when packing is on
 * (as_set_band_packing) and the pair's range proof holds for the class that
 * fits the request, else the 32-bit kernel (widths 64..1536).
 * lo_out/hi_out (device int32 [n_pairs], both or neither) receive the
 * diagonal limits actually computed, in A-rows/B-columns orientation
 * (j - i, j over B).  A request wider than 1536 diagonals returns AS_ERR_ARG.
 */
int as_band_scores(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                   const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                   const int32_t *band_w, int32_t *scores_out, int32_t *lo_out, int32_t *hi_out,
                   void *stream);

/*
 * Certified score of one exact band: the optimal score of pair p restricted
 * to the diagonals min(0, n-m) - w <= j - i <= max(0, n-m) + w themselves,
 * w = band_w[p] (no widening; |n - m| + 2w + 1 <= 1024 or AS_ERR_ARG), and
 * accept_out[p] = 1 when that score is at least the upper bound on every
 * path leaving those diagonals (then it is the optimal score), else 0.
 * A pair with band_w[p] < 0 is skipped: its outputs are left unchanged.
 * Pairs with an empty sequence are scored by their closed form and their
 * accept_out entry is left unchanged.
 *   band_w, scores_out, accept_out : device, int32 [n_pairs]
 * Same modes, alphabets and errors as as_align_batch_band.
 */
int as_band_certify(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                    const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                    const int32_t *band_w, int32_t *scores_out, int32_t *accept_out, void *stream);

/*
 * Learned band (the learned-band extension; not in the paper).  A small
 * network reads cheap per-pair features and predicts the initial half-width
 * of the certified banded path above, so every score stays exact whatever it
 * predicts; a good prediction only saves work.
 *
 * Network: 32 -> 64 -> 64 -> 1 with ReLU, y = log2(w + 1), float32
 * parameters in one device array of AS_MLP_PARAMS floats laid out as
 *   w1[32][64] (input-major), b1[64], w2[64][64], b2[64], w3[64], b3[1].
 * Products run on the matrix cores with operands rounded to bfloat16
 * (nearest even) and float32 accumulation; biases, ReLU, loss and optimiser
 * are float32.  The predicted half-width is ceil(2^y - 1) clamped to
 * [0, 2^20].
 */
#define AS_FEATURES 32
#define AS_MLP_PARAMS 6337
#define AS_BAND_WIDE 1024 /* label: no band of at most 1024 diagonals is accepted */

/*
 * Features of every pair (residues 0..3 only, else AS_ERR_RESIDUE):
 * 7-mers of A are looked up among the 7-mers of B that occur exactly once
 * (and start before position 65535); each hit at (i, j) adds one to signed
 * log2 bin b = min(14, floor(log2(1 + |d|))) of d = (j - i) -
 * trunc(i (n - m) / m): bin 15 + b for d >= 0, 14 - b otherwise.
 *   features_out[p][0..29] = bin counts / max(1, hits)
 *   features_out[p][30]    = log2(1 + |n - m|) / 16
 *   features_out[p][31]    = hits / max(1, m - 6)
 * features_out: device float [n_pairs][32], 16-byte aligned.
 */
int as_pair_features(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                     const int64_t *offs_b, int64_t n_pairs, float *features_out, void *stream);

/*
 * Network inference: band_w_out[p] = ceil(2^y_p - 1) clamped to [0, 2^20];
 * y_out (optional, NULL) receives y_p.  params, features (16-byte aligned),
 * band_w_out, y_out: device.
 */
int as_band_predict(const float *params, const float *features, int64_t n, int32_t *band_w_out,
                    float *y_out, void *stream);

/*
 * Band labels from the full DP: label_p is the smallest w >= 0 whose exact
 * band (as in as_band_certify) is accepted, when |n - m| + 2w + 1 <= 1024;
 * otherwise AS_BAND_WIDE.  The full-DP score S gives the search its lower
 * end (no band below the smallest w whose leave bound is <= S can be
 * accepted); exact bands are then tried with doubling and bisection.
 * Pairs with an empty sequence get 0.  Global and semi-global only.
 *   labels_out : device int32 [n_pairs]
 */
int as_band_labels(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                   const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                   int32_t *labels_out, void *stream);

/*
 * Adam training of the network, n_steps minibatches of `batch` samples:
 * step s uses samples order[s * batch .. s * batch + batch - 1] (indices
 * into features/labels, 0 <= index < n), target log2(label + 1), pinball
 * loss with quantile tau (0 < tau < 1), averaged over the minibatch, and
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) with step
 * counter t0 + s for the bias corrections.
 *   params, adam_m, adam_v : device float [AS_MLP_PARAMS], updated in place
 *                            (adam_m, adam_v zero before the first step)
 *   features : device float [n][32] (16-byte aligned); labels : device int32 [n] (>= 0)
 *   order    : device int32 [n_steps * batch]
 *   grads_out: optional device float [AS_MLP_PARAMS]: the first step's gradient
 * Out-of-range indices or negative labels return AS_ERR_ARG before any step.
 */
int as_band_train(float *params, float *adam_m, float *adam_v, const float *features,
                  const int32_t *labels, int64_t n, const int32_t *order, int32_t n_steps,
                  int32_t batch, int32_t t0, float lr, float tau, float *grads_out, void *stream);

/*
 * Features, labels and training in one call: params (device, AS_MLP_PARAMS
 * floats) hold the initial weights on entry and the trained ones on return;
 * order as in as_band_train (indices into this batch of pairs).
 */
int as_train_band_model(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                        const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                        int32_t mode, float *params, const int32_t *order, int32_t n_steps,
                        int32_t batch, float lr, float tau, void *stream);

/*
 * Versioned storage of a band network (not in the paper): its parameters
 * and, optionally, the Adam moments, so training can be resumed and a
 * trained network reused in another process.  The blob is host memory the
 * caller owns: a 64-byte header (magic "ASBANDMD", format version 1, the
 * parameter count, input and hidden sizes, whether Adam moments follow, the
 * Adam step counter, an FNV-1a checksum of the payload) and the float32
 * parameters in this library's layout, then the two moments.
 * as_band_model_blob_size(with_adam) is the exact size.  Save copies from
 * device memory (params, and adam_m / adam_v together or not at all);
 * *blob_size (optional) receives the size; a blob_cap below it returns
 * AS_ERR_ARG.  Load checks the magic, version, sizes and checksum
 * (AS_ERR_ARG on any mismatch), then copies into device memory; asking for
 * Adam moments from a blob without them returns AS_ERR_ARG.  Both wait for
 * their copies before returning.
 */
int64_t as_band_model_blob_size(int32_t with_adam);
int as_band_model_save(const float *params, const float *adam_m, const float *adam_v, int64_t adam_t,
                       void *blob_out, int64_t blob_cap, int64_t *blob_size, void *stream);
int as_band_model_load(const void *blob, int64_t blob_size, float *params_out, float *adam_m_out,
                       float *adam_v_out, int64_t *adam_t_out, void *stream);

/*
 * Learned-band alignment: features, network inference, then
 * as_align_batch_band with the predicted half-widths.  Every score is exact.
 * Same modes, alphabets and errors as as_align_batch_band, plus residues
 * above 3 (AS_ERR_RESIDUE).
 */
int as_align_batch_learned(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                           const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring,
                           int32_t mode, const float *params, int32_t max_rounds,
                           int32_t *scores_out, as_band_stats *stats, void *stream);

/*
 * Full-DP kernel variants per length bin (batching runtime; not in the
 * paper).  Bin b holds the pairs whose longer sequence has at most 64 << b
 * residues (b = 0..AS_LEN_BINS-1, the last bin everything longer).  Within
 * each kernel's work list the pairs are ordered by bin, longest first.  A
 * bin's variant is one of
 *   AS_VARIANT_AUTO       automatic: packed 16-bit when the shorter side has
 *                         at most 256 residues and the range is proven (or
 *                         local), the wavefront for at least 2048 rows and
 *                         more than one wavefront stripe (1024 columns; 512
 *                         for alphabets of more than 4 letters), else
 *                         AS_VARIANT_PACKED_LDS for local pairs whose
 *                         sigma + alpha fits a byte and 32-bit with K = 16
 *                         for the others;
 *   AS_VARIANT_PACKED16   packed 16-bit kernel (two pairs per lane group);
 *   AS_VARIANT_K8/K16/K32 32-bit stripe kernel with 8/16/32 columns per lane;
 *   AS_VARIANT_WAVEFRONT  multi-wave wavefront;
 *   AS_VARIANT_PACKED_LDS local mode: packed 16-bit cells in 128-column
 *                         stripes, two pairs per lane group, int8 profiles
 *                         of any alphabet in LDS; a pair whose 16-bit maximum
 *                         saturates is recomputed with 32-bit cells.
 * A pair the bin's variant cannot serve (packed: range or width; wavefront:
 * at most one stripe of columns; packed LDS: other modes) takes the
 * automatic rule.  Every variant computes
 * the same exact scores; the table only changes speed.  Tables are kept per
 * mode for the process.
 */
#define AS_LEN_BINS 12
#define AS_VARIANT_AUTO (-1)
#define AS_VARIANT_PACKED16 0
#define AS_VARIANT_K8 1
#define AS_VARIANT_K16 2
#define AS_VARIANT_K32 3
#define AS_VARIANT_WAVEFRONT 4
#define AS_VARIANT_PACKED_LDS 5
#define AS_VARIANTS 6

/* Set the table of a mode (HOST int8 [AS_LEN_BINS]; NULL: all automatic). */
int as_set_variants(int32_t mode, const int8_t *table);
/* Copy the table of a mode into table_out (HOST int8 [AS_LEN_BINS]). */
int as_get_variants(int32_t mode, int8_t *table_out);

/*
 * Persisted tables (the batching runtime's autotuner output, not in the
 * paper): the three modes' variant tables and measured cell types
 * (as_half_cells_preference) as one versioned, checksummed blob of
 * as_variant_tables_blob_size() bytes (68), host memory owned by the
 * caller.  Layout (little-endian): char magic[8] = "ASVARTAB"; uint32
 * version = 2, n_modes = 3, n_bins = AS_LEN_BINS, n_variants = AS_VARIANTS;
 * int8 table[3][AS_LEN_BINS]; int8 half_pref[3]; uint8 0; uint32 FNV-1a
 * checksum of the 68 bytes with this field zero.  A version-1 blob (64
 * bytes: no half_pref, the checksum at byte 60) still loads and clears the
 * measured cell types.  Save: AS_ERR_NULL, or AS_ERR_ARG when blob_size is
 * too small.  Load: a wrong size, magic, version, dimension, checksum or
 * entry returns AS_ERR_ARG and leaves every table as it was; otherwise all
 * three tables and cell types are replaced.
 */
int64_t as_variant_tables_blob_size(void);
int as_variant_tables_save(uint8_t *blob_out, int64_t blob_size);
int as_variant_tables_load(const uint8_t *blob, int64_t blob_size);

/*
 * Autotuner: for every length bin present in the batch, time each variant
 * on a sample of the bin's pairs (every stride-th pair: at most sample_pairs
 * pairs and about 1e11 cells; best of two runs, HIP events around the DP
 * kernels) and keep the fastest in the mode's table.  Bins without pairs
 * keep their entry.  Then, when the scoring admits FP16 cells
 * (as_set_half_cells) and a sampled bin can take the packed kernel, the
 * sampled bins run under the tuned table once with int16 and once with FP16
 * cells (best of two each), and the faster becomes the mode's measured cell
 * type (as_half_cells_preference).  The sample's scores go to library
 * scratch memory.
 *   gcups_out : optional HOST float [AS_LEN_BINS * AS_VARIANTS]: measured
 *               GCUPS per (bin, variant), 0 where not measured
 *   table_out : optional HOST int8 [AS_LEN_BINS]: the resulting table
 * Same arguments and errors as as_align_batch otherwise.
 */
int as_autotune(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                int32_t sample_pairs, float *gcups_out, int8_t *table_out, void *stream);

/*
 * Plans: one batch made replayable as a HIP graph (batching runtime).  A
 * plan binds the batch's device pointers, scoring, mode and scores_out, and
 * the mode's variant table at creation; it owns a private workspace sized by
 * a planning run, and every replay (as_plan_run) runs the whole pipeline --
 * classification, all DP kernels on persistent grids, the 32-bit re-run --
 * as one graph launch on `stream`, then waits for it and returns the status.
 * The caller may change the batch's contents between replays (same
 * pointers and pair count); a replay whose routing needs more boundary
 * memory than the plan holds returns AS_ERR_ARG without touching memory
 * beyond its buffers.  Calls on one plan must not overlap.
 */
typedef struct as_plan as_plan;
int as_plan_create(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                   const int64_t *offs_b, int64_t n_pairs, const as_scoring *scoring, int32_t mode,
                   int32_t *scores_out, as_plan **plan_out, void *stream);
int as_plan_run(as_plan *plan, void *stream);
int as_plan_destroy(as_plan *plan);

/*
 * Packed 16-bit banded kernel (global mode): a pair whose band cells are
 * proven to fit an unsigned 16-bit number with a per-pair bias is banded two
 * pairs per lane group with 16-bit cells, in widths of 80 to 1536 diagonals;
 * the others use the 32-bit banded kernel.  The proof, for an m x n pair and
 * a band of W diagonals, with UB = max(sigma_max, 0)*min(m,n) +
 * beta*(m + n + W) + alpha + 2*beta + 256 and LB = max(0, -(sigma_min +
 * 2*beta))*min(m,n) + 3*(alpha - beta) + 256: LB < 32000 and UB + LB < 65000.
 * On by default (certified rounds and as_band_scores; as_band_certify and
 * the labels always use 32-bit cells); on = 0 sends every pair to the
 * 32-bit kernel (scores are the same either way).  Returns the previous
 * setting.
 */
int as_set_band_packing(int32_t on);

/*
 * Saturation threshold of the packed 16-bit local path: a pair whose 16-bit
 * maximum reaches `limit` is treated as saturated and recomputed with 32-bit
 * cells.  The default, 32767, is the int16 saturation value itself; a lower
 * value only sends more pairs to the exact 32-bit re-run, which lets tests
 * force that path from the host.  limit <= 0 restores the default.
 * Returns the previous threshold.
 */
int as_set_i16_limit(int32_t limit);

/*
 * Cell type of the packed full-DP kernel (section 3.2: two alignments per
 * 32-bit register; the paper packs two FP16 values).  FP16 holds integers
 * exactly only up to 2048 in magnitude, so FP16 cells are used only for
 * calls whose sigma + bias and padding values all lie in 0..16 (bias =
 * alpha for local, alpha + beta otherwise), and under them the packed
 * kernel takes only global and semi-global pairs with
 * sigma_max*256 + beta*(rows + 512) + alpha + 2*beta + 16 < 1984 (the
 * others take the 32-bit kernels); local pairs whose FP16 maximum reaches
 * 1984 are recomputed with 32-bit cells.  Scores are identical under every
 * setting.
 *   mode 0: int16 cells always.
 *   mode 1: FP16 cells for every call that admits them.
 *   mode 2 (default, any other value): FP16 cells for local calls whose
 *           profile values are exact in FP8 E5M2 (0..8, 10, 12, 14, 16) and
 *           whose maxima cannot reach 1984 (sigma_max*256 + alpha + 16 <
 *           1984), int16 otherwise; as_align_all_vs_all also takes them for
 *           global and semi-global calls with E5M2-exact values whose
 *           longest row sequence satisfies the bound above.
 *           A measured cell type for the mode (as_half_cells_preference,
 *           set by as_autotune) replaces this rule for as_align_batch and
 *           plans.
 * Applies to calls and plans made after it.  Returns the previous mode.
 */
int as_set_half_cells(int mode);

/*
 * The automatic setting's measured cell type for a mode (batching runtime;
 * not in the paper): -1 none (the static rule of as_set_half_cells mode 2
 * decides), 0 int16, 1 FP16 cells where the scoring admits them.
 * as_autotune sets it; set != 0 stores pref (-1, 0 or 1), set == 0 only
 * reads.  Returns the previous value, or AS_ERR_ARG for a mode outside 0..2
 * or such a pref.  Per process, for calls and plans made after it.
 */
int as_half_cells_preference(int32_t mode, int32_t pref, int32_t set);

/* Enable (1) or disable (0) phase timing.  Returns the previous setting. */
int as_enable_timing(int on);
/* Copy the last call's phase times into *out (host).  AS_ERR_NULL if out is NULL. */
int as_last_timing(as_timing *out);

#ifdef __cplusplus
}
#endif

#endif /* ANYSEQ_MI_H */
