"""Pins of the oracle's alignments (the paper's "Traceback" paragraph of
section 2.1: the optimal score is reached by an actual alignment found by
tracing predecessors back).  The alignment scorer is pinned by hand-worked
alignments and by the brute-force enumeration of every alignment of tiny
pairs (scored column by column in tests/brute.py); the traceback is pinned
by the scorer and the optimal score: every traced alignment is admitted by
its mode and scores exactly the DP optimum."""
import numpy as np
import pytest

import brute
from oracle import GLOBAL, LOCAL, SEMIGLOBAL

DNA = np.full((4, 4), -3, dtype=np.int8)
np.fill_diagonal(DNA, 2)


def _enc(x):
    return ["ACGT".index(c) for c in x]


def _random_scoring(rng, asz):
    sub = rng.integers(-4, 1, size=(asz, asz))
    sub[np.arange(asz), np.arange(asz)] = rng.integers(1, 4, size=asz)
    sub = sub + np.triu(rng.integers(0, 2, size=(asz, asz)), 1)   # not symmetric
    beta = int(rng.integers(0, 4))
    alpha = beta + int(rng.integers(0, 5))
    return sub.astype(np.int8), alpha, beta


def test_alignment_score_worked_examples(oracle_mod):
    sc = oracle_mod.alignment_score
    # ACGT / AC-T: +2 +2 -5 +2
    assert sc(_enc("ACGT"), _enc("ACT"), DNA, 5, 2, GLOBAL, "MMIM", (0, 4, 0, 3)) == 1
    # AAAATTTT / AAAA----: 8 - (5 + 3*2); with linear gaps alpha = beta = 2: 8 - 8
    assert sc(_enc("AAAATTTT"), _enc("AAAA"), DNA, 5, 2, GLOBAL, "MMMMIIII", (0, 8, 0, 4)) == -3
    assert sc(_enc("AAAATTTT"), _enc("AAAA"), DNA, 2, 2, GLOBAL, "MMMMIIII", (0, 8, 0, 4)) == 0
    # one gap run split by a match is two runs; an I run next to a D run is two runs
    assert sc(_enc("AAAA"), _enc("AA"), DNA, 5, 2, GLOBAL, "IMIM", (0, 4, 0, 2)) == 4 - 10
    assert sc(_enc("AC"), _enc("GT"), DNA, 5, 2, GLOBAL, "IIDD", (0, 2, 0, 2)) == -7 - 7
    assert sc([], _enc("ACG"), DNA, 5, 2, GLOBAL, "DDD", (0, 0, 0, 3)) == -9
    # semi-global CA / GA: aligning the two A's would cut off both prefixes
    assert sc(_enc("CA"), _enc("GA"), DNA, 5, 2, SEMIGLOBAL, "", (2, 2, 0, 0)) == 0
    assert sc(_enc("CA"), _enc("GA"), DNA, 5, 2, SEMIGLOBAL, "M", (1, 2, 1, 2)) == oracle_mod.INVALID
    # ACGT inside TTACGTTT: free end gaps of the longer sequence
    assert sc(_enc("ACGT"), _enc("TTACGTTT"), DNA, 5, 2, SEMIGLOBAL, "MMMM", (0, 4, 2, 6)) == 8
    # local: any substrings, the empty alignment included
    assert sc(_enc("TTACGTAA"), _enc("GGACGTCC"), DNA, 5, 2, LOCAL, "MMMM", (2, 6, 2, 6)) == 8
    assert sc(_enc("TTACGTAA"), _enc("GGACGTCC"), DNA, 5, 2, LOCAL, "", (3, 3, 5, 5)) == 0


def test_alignment_score_rejects(oracle_mod):
    sc, bad = oracle_mod.alignment_score, oracle_mod.INVALID
    q, s = _enc("ACGT"), _enc("ACT")
    assert sc(q, s, DNA, 5, 2, GLOBAL, "MMM", (0, 4, 0, 3)) == bad         # A not consumed
    assert sc(q, s, DNA, 5, 2, GLOBAL, "MMMM", (0, 4, 0, 3)) == bad        # runs past B
    assert sc(q, s, DNA, 5, 2, GLOBAL, "MMM", (0, 3, 0, 3)) == bad         # global needs all of A
    assert sc(q, s, DNA, 5, 2, GLOBAL, "MMXM", (0, 4, 0, 3)) == bad        # unknown column
    assert sc(q, s, DNA, 5, 2, SEMIGLOBAL, "MM", (1, 3, 1, 3)) == bad      # both prefixes cut
    assert sc(q, s, DNA, 5, 2, SEMIGLOBAL, "M", (0, 1, 0, 1)) == bad       # both suffixes cut
    assert sc(q, s, DNA, 5, 2, LOCAL, "M", (3, 4, 2, 4)) == bad            # span/columns disagree
    assert sc(q, s, DNA, 5, 2, LOCAL, "M", (3, 5, 2, 3)) == bad            # span past A


def test_alignment_score_equals_enumeration(oracle_mod):
    """Every alignment of random tiny pairs: the scorer's value equals the
    enumeration's column-by-column score (global on whole sequences, local on
    the substrings), and the best of them is the DP optimum."""
    rng = np.random.default_rng(2101)
    n_checked = 0
    for _ in range(40):
        sub, alpha, beta = _random_scoring(rng, 3)
        q = rng.integers(0, 3, size=int(rng.integers(0, 5))).tolist()
        s = rng.integers(0, 3, size=int(rng.integers(0, 5))).tolist()
        alns = brute.all_alignments(q, s, sub, alpha, beta)
        for cols, score in alns:
            assert oracle_mod.alignment_score(q, s, sub, alpha, beta, GLOBAL, cols,
                                              (0, len(q), 0, len(s))) == score
            n_checked += 1
        assert max(x[1] for x in alns) == oracle_mod.align_pair(q, s, sub, alpha, beta, GLOBAL)
        # a substring pair, scored as a local alignment
        a0 = int(rng.integers(0, len(q) + 1)); a1 = int(rng.integers(a0, len(q) + 1))
        b0 = int(rng.integers(0, len(s) + 1)); b1 = int(rng.integers(b0, len(s) + 1))
        for cols, score in brute.all_alignments(q[a0:a1], s[b0:b1], sub, alpha, beta):
            assert oracle_mod.alignment_score(q, s, sub, alpha, beta, LOCAL, cols,
                                              (a0, a1, b0, b1)) == score
    assert n_checked > 500


@pytest.mark.parametrize("mode", [GLOBAL, SEMIGLOBAL, LOCAL])
def test_traceback_is_optimal_alignment(oracle_mod, mode):
    """The traced alignment is admitted by the mode and scores exactly the
    optimum: on tiny pairs with random non-symmetric scoring (0 <= beta <=
    alpha, linear gaps included) and on short related DNA pairs."""
    rng = np.random.default_rng(2200 + mode)
    cases = []
    for _ in range(150):
        sub, alpha, beta = _random_scoring(rng, 3)
        q = rng.integers(0, 3, size=int(rng.integers(0, 8))).tolist()
        s = rng.integers(0, 3, size=int(rng.integers(0, 8))).tolist()
        cases.append((q, s, sub, alpha, beta))
    for _ in range(60):
        a = rng.integers(0, 4, size=int(rng.integers(1, 120))).tolist()
        b = list(a)
        for _k in range(int(rng.integers(0, 12))):
            pos = int(rng.integers(0, len(b)))
            r = rng.random()
            if r < 0.3 and len(b) > 1:
                del b[pos]
            elif r < 0.6:
                b.insert(pos, int(rng.integers(0, 4)))
            else:
                b[pos] = int(rng.integers(0, 4))
        cases.append((a, b, DNA, 5, 2))
    for q, s, sub, alpha, beta in cases:
        score, cols, span = oracle_mod.traceback_pair(q, s, sub, alpha, beta, mode)
        assert score == oracle_mod.align_pair(q, s, sub, alpha, beta, mode)
        assert oracle_mod.alignment_score(q, s, sub, alpha, beta, mode, cols, span) == score, \
            (q, s, cols, span)


def test_traceback_worked_examples(oracle_mod):
    """Pairs of the worked-example table whose optimal alignment is unique."""
    tb = oracle_mod.traceback_pair
    assert tb(_enc("ACGT"), _enc("ACT"), DNA, 5, 2, GLOBAL) == (1, "MMIM", (0, 4, 0, 3))
    assert tb([], _enc("ACG"), DNA, 5, 2, GLOBAL) == (-9, "DDD", (0, 0, 0, 3))
    assert tb(_enc("TTACGTAA"), _enc("GGACGTCC"), DNA, 5, 2, LOCAL) == (8, "MMMM", (2, 6, 2, 6))
    assert tb(_enc("ACGT"), _enc("TTACGTTT"), DNA, 5, 2, SEMIGLOBAL) == (8, "MMMM", (0, 4, 2, 6))


def test_batch_drivers(oracle_mod):
    from paper_2205_07610_amd import synth
    rng = np.random.default_rng(2300)
    sa, oa, sb, ob = synth.random_small(rng, 300, 90, related=0.7)
    for mode in (GLOBAL, SEMIGLOBAL, LOCAL):
        sc, ops, span = oracle_mod.traceback_batch(sa, oa, sb, ob, DNA, 5, 2, mode)
        assert np.array_equal(sc, oracle_mod.align_batch(sa, oa, sb, ob, DNA, 5, 2, mode))
        again = oracle_mod.alignment_score_batch(sa, oa, sb, ob, DNA, 5, 2, mode, ops, span)
        assert np.array_equal(again, sc)
        for p in range(0, 300, 37):
            q, s = sa[oa[p]:oa[p + 1]], sb[ob[p]:ob[p + 1]]
            start = int(oa[p] - oa[0] + ob[p] - ob[0])
            one = oracle_mod.traceback_pair(q, s, DNA, 5, 2, mode)
            assert ops[start:start + span[p][0]].tobytes().decode() == one[1]
            assert tuple(span[p][1:]) == one[2]
        # a corrupted alignment is caught
        k = int(np.nonzero(span[:, 0] > 2)[0][0])
        start = int(oa[k] - oa[0] + ob[k] - ob[0])
        bad = ops.copy()
        bad[start] = ord("I") if bad[start] != ord("I") else ord("D")
        got = oracle_mod.alignment_score_batch(sa, oa, sb, ob, DNA, 5, 2, mode, bad, span)
        assert got[k] == oracle_mod.INVALID or got[k] < sc[k]
