"""Pins for the CPU oracle: each test checks it against something other than
itself -- hand-computed examples, brute-force enumeration of alignments,
closed forms of classic special cases, and invariants of the definitions.

The brute-force tests use random, NON-symmetric substitution matrices, so a
transposed sigma lookup, a dropped E/F term, a wrong gap-open/extend order or
a wrong boundary row all fail at least one of them.
"""
import os

import numpy as np
import pytest

import brute
from oracle import GLOBAL, LOCAL, SEMIGLOBAL

pytestmark = pytest.mark.filterwarnings("ignore")

ENC = {"A": 0, "C": 1, "G": 2, "T": 3}
MODES = {"global": GLOBAL, "semiglobal": SEMIGLOBAL, "local": LOCAL}
DNA = np.full((4, 4), -3, dtype=np.int8)
np.fill_diagonal(DNA, 2)


def _enc(s):
    return [] if s == "-" else [ENC[c] for c in s]


def _golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = line.split()
        rows.append((f[0], f[1], MODES[f[2]], int(f[3]), int(f[4]), int(f[5])))
    return rows


@pytest.mark.parametrize("q,s,mode,alpha,beta,expected", _golden())
def test_worked_examples(oracle_mod, q, s, mode, alpha, beta, expected):
    assert oracle_mod.align_pair(_enc(q), _enc(s), DNA, alpha, beta, mode) == expected


def _random_scoring(rng, asz):
    sub = rng.integers(-4, 1, size=(asz, asz))
    sub[np.arange(asz), np.arange(asz)] = rng.integers(1, 4, size=asz)
    # break symmetry on purpose so a transposed lookup cannot pass
    sub = sub + np.triu(rng.integers(0, 2, size=(asz, asz)), 1)
    beta = int(rng.integers(0, 4))
    alpha = beta + int(rng.integers(0, 5))
    return sub.astype(np.int8), alpha, beta


def test_brute_force_global(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(250):
        asz = int(rng.integers(2, 5))
        sub, alpha, beta = _random_scoring(rng, asz)
        q = rng.integers(0, asz, size=int(rng.integers(0, 7))).tolist()
        s = rng.integers(0, asz, size=int(rng.integers(0, 7))).tolist()
        want = brute.global_score(q, s, sub, alpha, beta)
        assert oracle_mod.align_pair(q, s, sub, alpha, beta, GLOBAL) == want, (q, s, sub, alpha, beta)


@pytest.mark.parametrize("mode", [SEMIGLOBAL, LOCAL])
def test_brute_force_local_semiglobal(oracle_mod, mode):
    rng = np.random.default_rng(12 + mode)
    for _ in range(80):
        asz = int(rng.integers(2, 5))
        sub, alpha, beta = _random_scoring(rng, asz)
        q = rng.integers(0, asz, size=int(rng.integers(0, 6))).tolist()
        s = rng.integers(0, asz, size=int(rng.integers(0, 6))).tolist()
        want = brute.SCORERS[mode](q, s, sub, alpha, beta)
        got = oracle_mod.align_pair(q, s, sub, alpha, beta, mode)
        assert got == want, (mode, q, s, sub, alpha, beta)


# ---- closed forms ---------------------------------------------------------

def _levenshtein(a, b):
    """Textbook edit distance (unit substitution / insertion / deletion)."""
    prev = list(range(len(b) + 1))
    for i, x in enumerate(a, 1):
        cur = [i]
        for j, y in enumerate(b, 1):
            cur.append(min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (x != y)))
        prev = cur
    return prev[-1]


def _lcs(a, b):
    """Textbook longest common subsequence length."""
    prev = [0] * (len(b) + 1)
    for x in a:
        cur = [0]
        for j, y in enumerate(b, 1):
            cur.append(prev[j - 1] + 1 if x == y else max(prev[j], cur[j - 1]))
        prev = cur
    return prev[-1]


def _longest_common_substring(a, b):
    best = 0
    for i in range(len(a)):
        for j in range(len(b)):
            k = 0
            while i + k < len(a) and j + k < len(b) and a[i + k] == b[j + k]:
                k += 1
            best = max(best, k)
    return best


def _longest_exact_overlap(a, b):
    """Longest exact match that runs from a start boundary to an end boundary:
    a suffix of one sequence equal to a prefix of the other, or one sequence
    contained in the other."""
    best = 0
    m, n = len(a), len(b)
    for off in range(-m, n + 1):          # diagonal j - i = off
        i0, j0 = max(0, -off), max(0, off)
        length = min(m - i0, n - j0)
        if length > 0 and list(a[i0:i0 + length]) == list(b[j0:j0 + length]):
            best = max(best, length)
    return best


def test_closed_form_levenshtein(oracle_mod):
    rng = np.random.default_rng(21)
    sub = np.full((4, 4), -1, dtype=np.int8)
    np.fill_diagonal(sub, 0)
    for _ in range(60):
        a = rng.integers(0, 4, size=int(rng.integers(0, 60))).tolist()
        b = rng.integers(0, 4, size=int(rng.integers(0, 60))).tolist()
        assert oracle_mod.align_pair(a, b, sub, 1, 1, GLOBAL) == -_levenshtein(a, b)


def test_closed_form_lcs(oracle_mod):
    rng = np.random.default_rng(22)
    sub = np.full((4, 4), -2, dtype=np.int8)
    np.fill_diagonal(sub, 2)
    for _ in range(60):
        a = rng.integers(0, 4, size=int(rng.integers(0, 60))).tolist()
        b = rng.integers(0, 4, size=int(rng.integers(0, 60))).tolist()
        assert oracle_mod.align_pair(a, b, sub, 1, 1, GLOBAL) == 4 * _lcs(a, b) - len(a) - len(b)


def test_closed_form_local_common_substring(oracle_mod):
    rng = np.random.default_rng(23)
    sub = np.full((4, 4), -50, dtype=np.int8)
    np.fill_diagonal(sub, 1)
    for _ in range(60):
        a = rng.integers(0, 4, size=int(rng.integers(0, 40))).tolist()
        b = rng.integers(0, 4, size=int(rng.integers(0, 40))).tolist()
        assert oracle_mod.align_pair(a, b, sub, 50, 50, LOCAL) == _longest_common_substring(a, b)


def test_closed_form_semiglobal_exact_overlap(oracle_mod):
    rng = np.random.default_rng(24)
    sub = np.full((4, 4), -50, dtype=np.int8)
    np.fill_diagonal(sub, 1)
    for _ in range(80):
        a = rng.integers(0, 2, size=int(rng.integers(0, 30))).tolist()
        b = rng.integers(0, 2, size=int(rng.integers(0, 30))).tolist()
        assert oracle_mod.align_pair(a, b, sub, 50, 50, SEMIGLOBAL) == _longest_exact_overlap(a, b)


def test_empty_sequences(oracle_mod):
    for n in range(0, 8):
        s = [1] * n
        for alpha, beta in [(5, 2), (3, 3), (0, 0), (7, 1)]:
            want = 0 if n == 0 else -alpha - beta * (n - 1)
            assert oracle_mod.align_pair([], s, DNA, alpha, beta, GLOBAL) == want
            assert oracle_mod.align_pair(s, [], DNA, alpha, beta, GLOBAL) == want
            for mode in (SEMIGLOBAL, LOCAL):
                assert oracle_mod.align_pair([], s, DNA, alpha, beta, mode) == 0
                assert oracle_mod.align_pair(s, [], DNA, alpha, beta, mode) == 0


def test_identical_sequences(oracle_mod):
    rng = np.random.default_rng(25)
    for n in (1, 17, 150, 400):
        a = rng.integers(0, 4, size=n).tolist()
        for mode in (GLOBAL, SEMIGLOBAL, LOCAL):
            assert oracle_mod.align_pair(a, a, DNA, 5, 2, mode) == 2 * n


# ---- invariants -------------------------------------------------------------

def test_invariants(oracle_mod):
    rng = np.random.default_rng(31)
    sub = np.full((4, 4), -3, dtype=np.int8)
    np.fill_diagonal(sub, 2)
    for _ in range(150):
        a = rng.integers(0, 4, size=int(rng.integers(0, 50))).tolist()
        b = rng.integers(0, 4, size=int(rng.integers(0, 50))).tolist()
        beta = int(rng.integers(0, 4))
        alpha = beta + int(rng.integers(0, 6))
        sc = {md: oracle_mod.align_pair(a, b, sub, alpha, beta, md) for md in (GLOBAL, SEMIGLOBAL, LOCAL)}
        assert sc[LOCAL] >= sc[SEMIGLOBAL] >= sc[GLOBAL]
        assert sc[LOCAL] >= 0 and sc[SEMIGLOBAL] >= 0
        for md in (GLOBAL, SEMIGLOBAL, LOCAL):
            # symmetric sigma: swapping the sequences is a transposition
            assert oracle_mod.align_pair(b, a, sub, alpha, beta, md) == sc[md]
            # reversing both sequences reverses every alignment
            assert oracle_mod.align_pair(a[::-1], b[::-1], sub, alpha, beta, md) == sc[md]


def test_transpose_nonsymmetric_sigma(oracle_mod):
    rng = np.random.default_rng(32)
    for _ in range(60):
        sub, alpha, beta = _random_scoring(rng, 4)
        a = rng.integers(0, 4, size=int(rng.integers(0, 30))).tolist()
        b = rng.integers(0, 4, size=int(rng.integers(0, 30))).tolist()
        for md in (GLOBAL, SEMIGLOBAL, LOCAL):
            assert (oracle_mod.align_pair(a, b, sub, alpha, beta, md)
                    == oracle_mod.align_pair(b, a, sub.T.copy(), alpha, beta, md))


def test_batch_matches_pairs(oracle_mod):
    from paper_2205_07610_amd import synth
    b = synth.config0(n_pairs=40)
    got = oracle_mod.align_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, b.subst, b.alpha, b.beta,
                                 b.mode, nthreads=3)
    for p in range(b.n_pairs):
        q, s = b.pair(p)
        assert got[p] == oracle_mod.align_pair(q, s, b.subst, b.alpha, b.beta, b.mode)


# ---- band -------------------------------------------------------------------

def _band_ok(m, n, w):
    lo, hi = min(0, n - m) - w, max(0, n - m) + w
    return lambda i, j: lo <= j - i <= hi


@pytest.mark.parametrize("mode", [GLOBAL, SEMIGLOBAL, LOCAL])
def test_banded_brute_force(oracle_mod, mode):
    rng = np.random.default_rng(41 + mode)
    for _ in range(60 if mode == GLOBAL else 25):
        sub, alpha, beta = _random_scoring(rng, 3)
        q = rng.integers(0, 3, size=int(rng.integers(0, 6))).tolist()
        s = rng.integers(0, 3, size=int(rng.integers(0, 6))).tolist()
        w = int(rng.integers(0, 4))
        want = brute.SCORERS[mode](q, s, sub, alpha, beta, cell_ok=_band_ok(len(q), len(s), w))
        got = oracle_mod.banded_pair(q, s, sub, alpha, beta, mode, w)
        if want == float("-inf"):
            assert got <= -(1 << 59)
        else:
            assert got == want, (mode, q, s, w)


def test_banded_monotone_and_full(oracle_mod):
    rng = np.random.default_rng(45)
    for _ in range(40):
        a = rng.integers(0, 4, size=int(rng.integers(1, 60))).tolist()
        b = rng.integers(0, 4, size=int(rng.integers(1, 60))).tolist()
        for md in (GLOBAL, SEMIGLOBAL, LOCAL):
            full = oracle_mod.align_pair(a, b, DNA, 5, 2, md)
            prev = None
            for w in range(0, max(len(a), len(b)) + 2):
                v = oracle_mod.banded_pair(a, b, DNA, 5, 2, md, w)
                assert v <= full
                if prev is not None:
                    assert v >= prev
                prev = v
            assert prev == full


# ---- band acceptance bound: soundness by enumeration of band-leaving paths ----

@pytest.mark.parametrize("mode", [GLOBAL, SEMIGLOBAL])
def test_band_bound_sound(oracle_mod, mode):
    """Every path that leaves the band scores at most UB_out(w) (enumerated),
    and an accepted banded score equals the full score."""
    from oracle import band
    rng = np.random.default_rng(51 + mode)
    checked = 0
    for _ in range(70 if mode == GLOBAL else 30):
        sub, alpha, beta = _random_scoring(rng, 3)
        q = rng.integers(0, 3, size=int(rng.integers(0, 7 if mode == GLOBAL else 6))).tolist()
        s = rng.integers(0, 3, size=int(rng.integers(0, 7 if mode == GLOBAL else 6))).tolist()
        m, n = len(q), len(s)
        smax = int(sub.max())
        for w in range(0, max(m, n) + 1):
            ub = band.ub_outside(m, n, w, smax, alpha, beta, mode)
            out = brute.SCORERS[mode](q, s, sub, alpha, beta, cell_ok=_band_ok(m, n, w), escape=True)
            if ub is None:
                assert out == float("-inf"), (q, s, w)
                continue
            assert out <= ub, (mode, q, s, w, out, ub)
            checked += 1
            sb = oracle_mod.banded_pair(q, s, sub, alpha, beta, mode, w)
            if band.accepts(sb, ub):
                assert sb == oracle_mod.align_pair(q, s, sub, alpha, beta, mode)
    assert checked > (50 if mode == GLOBAL else 20)


def test_band_widths(oracle_mod):
    from oracle import band
    rng = np.random.default_rng(55)
    for _ in range(30):
        a = rng.integers(0, 4, size=int(rng.integers(1, 80))).tolist()
        b = list(a)
        for _k in range(int(rng.integers(0, 6))):     # a few edits
            pos = int(rng.integers(0, len(b) + 1))
            if rng.random() < 0.5 and len(b) > 1:
                del b[min(pos, len(b) - 1)]
            else:
                b.insert(pos, int(rng.integers(0, 4)))
        for md in (GLOBAL, SEMIGLOBAL):
            full = oracle_mod.align_pair(a, b, DNA, 5, 2, md)
            wa = band.accepted_width(a, b, DNA, 5, 2, md)
            we = band.exact_width(a, b, DNA, 5, 2, md)
            assert we <= wa
            assert oracle_mod.banded_pair(a, b, DNA, 5, 2, md, wa) == full
            assert oracle_mod.banded_pair(a, b, DNA, 5, 2, md, we) == full
            if we > 0:
                assert oracle_mod.banded_pair(a, b, DNA, 5, 2, md, we - 1) < full


def test_diag_band_matches_w_band_and_brute(oracle_mod):
    """Explicit diagonal limits reproduce the half-width band and brute force
    restricted to those diagonals (asymmetric limits included)."""
    from oracle import band
    rng = np.random.default_rng(61)
    for _ in range(60):
        sub, alpha, beta = _random_scoring(rng, 3)
        q = rng.integers(0, 3, size=int(rng.integers(0, 6))).tolist()
        s = rng.integers(0, 3, size=int(rng.integers(0, 6))).tolist()
        m, n = len(q), len(s)
        for mode in (GLOBAL, SEMIGLOBAL):
            w = int(rng.integers(0, 3))
            lo, hi = band.band_limits(m, n, w)
            assert (oracle_mod.diag_band_pair(q, s, sub, alpha, beta, mode, lo, hi)
                    == oracle_mod.banded_pair(q, s, sub, alpha, beta, mode, w))
            hi2 = hi + int(rng.integers(0, 4))
            lo2 = lo - int(rng.integers(0, 4))
            want = brute.SCORERS[mode](q, s, sub, alpha, beta,
                                       cell_ok=lambda i, j: lo2 <= j - i <= hi2)
            got = oracle_mod.diag_band_pair(q, s, sub, alpha, beta, mode, lo2, hi2)
            assert got == want or (want == float("-inf") and got <= -(1 << 59))
            ub = band.ub_outside_diag(m, n, lo2, hi2, int(sub.max()), alpha, beta, mode)
            out = brute.SCORERS[mode](q, s, sub, alpha, beta,
                                      cell_ok=lambda i, j: lo2 <= j - i <= hi2, escape=True)
            if ub is None:
                assert out == float("-inf")
            else:
                assert out <= ub


# ---- band acceptance bound: its value, pinned by enumeration ------------------

@pytest.mark.parametrize("mode", [GLOBAL, SEMIGLOBAL])
def test_band_bound_value_equals_best_leaving_path(oracle_mod, mode):
    """On one-letter pairs every diagonal step scores sigma_max, so the bound
    is attained: the best band-leaving path found by enumerating every
    alignment equals UB_out exactly (not merely stays below it).  A dropped
    gap run (-alpha instead of -2 alpha), a wrong count of gap columns (the
    -2 in beta*(m+n-2g-2)) or a wrong diagonal length in semi-global mode
    changes the value and fails here.  sigma ranges over negative values too,
    where the best leaving path takes no diagonal step at all."""
    from oracle import band
    rng = np.random.default_rng(91 + mode)
    checked = 0
    for sigma in (-4, -3, -1, 0, 1, 2, 3, 5):
        sub = np.array([[sigma]], dtype=np.int8)
        for _ in range(8 if mode == GLOBAL else 5):
            beta = int(rng.integers(0, 4))
            alpha = beta + int(rng.integers(0, 5))
            m = int(rng.integers(0, 7 if mode == GLOBAL else 6))
            n = int(rng.integers(0, 7 if mode == GLOBAL else 6))
            q, s = [0] * m, [0] * n
            for w in range(0, max(m, n) + 1):
                ub = band.ub_outside(m, n, w, sigma, alpha, beta, mode)
                out = brute.SCORERS[mode](q, s, sub, alpha, beta, cell_ok=_band_ok(m, n, w),
                                          escape=True)
                if ub is None:
                    assert out == float("-inf"), (m, n, w)
                    continue
                assert out == ub, (mode, sigma, alpha, beta, m, n, w, out, ub)
                checked += 1
    assert checked > (100 if mode == GLOBAL else 40)


def test_band_bound_closed_form_grid():
    """Global mode, sigma_max + 2 beta >= 0: the bound is the closed form
    sigma_max (min(m,n) - w - 1) - 2 alpha - beta (|n - m| + 2 w) of the
    corner-to-corner path with two gap runs (the best path off the band
    leaves it on either side with w + 1 gap columns and returns), on a grid
    of shapes, widths and scores; and no bound exists once the band holds
    every diagonal of the matrix."""
    from oracle import band
    for m in (1, 2, 5, 17, 40):
        for n in (1, 3, 17, 41, 90):
            for w in range(0, max(m, n) + 2, 3):
                for smax, alpha, beta in ((2, 5, 2), (1, 1, 1), (3, 11, 1), (5, 0, 0), (1, 7, 3)):
                    for mode in (GLOBAL, SEMIGLOBAL):
                        ub = band.ub_outside(m, n, w, smax, alpha, beta, mode)
                        lo, hi = band.band_limits(m, n, w)
                        if lo <= -m and hi >= n:
                            assert ub is None
                            continue
                        if mode == GLOBAL:
                            want = smax * (min(m, n) - w - 1) - 2 * alpha - beta * (abs(n - m) + 2 * w)
                        else:
                            # the longest diagonal just outside the band
                            lens = []
                            if hi + 1 <= n:
                                lens.append(min(m, n - hi - 1))
                            if lo - 1 >= -m:
                                lens.append(min(m + lo - 1, n))
                            want = smax * max(lens)
                        assert ub == want, (m, n, w, smax, alpha, beta, mode, ub, want)


def _accepted_by_scan(oracle_mod, a, b, sub, alpha, beta, mode):
    """Smallest accepted half-width by a plain scan upward from 0."""
    from oracle import band
    smax = int(np.asarray(sub).max())
    w = 0
    while True:
        sb = oracle_mod.banded_pair(a, b, sub, alpha, beta, mode, w)
        if band.accepts(sb, band.ub_outside(len(a), len(b), w, smax, alpha, beta, mode)):
            return w
        w += 1


@pytest.mark.parametrize("mode", [GLOBAL, SEMIGLOBAL])
def test_accepted_width_is_minimal(oracle_mod, mode):
    """The bisection's width is the smallest accepted one: it equals a linear
    scan from w = 0, and for wa > 0 the band of half-width wa - 1 is
    rejected.  Random tiny pairs (random scoring) and short related pairs
    (the benchmark scoring) cover rejected, accepted-at-zero and
    band-covers-everything cases."""
    from oracle import band
    rng = np.random.default_rng(97 + mode)
    positive = 0
    cases = []
    for _ in range(60):
        sub, alpha, beta = _random_scoring(rng, 3)
        q = rng.integers(0, 3, size=int(rng.integers(0, 9))).tolist()
        s = rng.integers(0, 3, size=int(rng.integers(0, 9))).tolist()
        cases.append((q, s, sub, alpha, beta))
    for _ in range(40):
        a = rng.integers(0, 4, size=int(rng.integers(5, 90))).tolist()
        b = list(a)
        for _k in range(int(rng.integers(0, 10))):
            pos = int(rng.integers(0, len(b)))
            r = rng.random()
            if r < 0.35 and len(b) > 1:
                del b[pos]
            elif r < 0.7:
                b.insert(pos, int(rng.integers(0, 4)))
            else:
                b[pos] = int(rng.integers(0, 4))
        cases.append((a, b, DNA, 5, 2))
    for q, s, sub, alpha, beta in cases:
        wa = band.accepted_width(q, s, sub, alpha, beta, mode)
        assert wa == _accepted_by_scan(oracle_mod, q, s, sub, alpha, beta, mode), (q, s)
        if wa > 0:
            positive += 1
            smax = int(np.asarray(sub).max())
            sb = oracle_mod.banded_pair(q, s, sub, alpha, beta, mode, wa - 1)
            assert not band.accepts(sb, band.ub_outside(len(q), len(s), wa - 1, smax, alpha, beta,
                                                        mode)), (q, s, wa)
    assert positive > 20
