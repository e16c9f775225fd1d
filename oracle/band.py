"""Band acceptance bound and band label -- TEST INFRASTRUCTURE ONLY.

The banded score S_band(w) keeps only cells with L <= j-i <= U,
L = min(0, n-m) - w, U = max(0, n-m) + w.  It equals the full score whenever
no path that leaves the band can beat it, so a banded score is accepted when
S_band(w) >= UB_out(w), an upper bound on every path that visits a cell off
the band.  The paper has no band; these bounds follow from the path
structure of its Eq. (1),(4),(5) (0 <= beta <= alpha assumed):

global -- a path from (0,0) to (m,n) that reaches diagonal U+1 takes at
least U+1 horizontal steps and U+1-(n-m) vertical ones (it must come back to
diagonal n-m); one reaching L-1 takes at least 1-L vertical and n-m-L+1
horizontal steps.  With g diagonal steps it has h+v = m+n-2g gap columns in
at least two runs, so its score is at most
    sigma_max*g - 2*alpha - beta*(m+n-2g-2),
maximised over 0 <= g <= (m+n-G)/2 where G is the side's minimum h+v.

semi-global -- any path through a cell of diagonal d has at most len(d)
diagonal steps (len(d) = min(m, n-d) for d >= 0, min(m+d, n) for d < 0) and
its gaps cost >= 0, so its score is at most
max(sigma_max, 0) * len(d); len is largest on the band's nearest outer
diagonals U+1 and L-1.

UB_out is None when no path can leave the band (accept unconditionally).
"""
from __future__ import annotations

from . import GLOBAL, SEMIGLOBAL, banded_pair, align_pair


def band_limits(m: int, n: int, w: int) -> tuple[int, int]:
    return min(0, n - m) - w, max(0, n - m) + w


def ub_outside(m: int, n: int, w: int, sigma_max: int, alpha: int, beta: int, mode: int):
    lo, hi = band_limits(m, n, w)
    return ub_outside_diag(m, n, lo, hi, sigma_max, alpha, beta, mode)


def ub_outside_diag(m: int, n: int, lo: int, hi: int, sigma_max: int, alpha: int, beta: int,
                    mode: int):
    """Upper bound on every path that visits a diagonal outside [lo, hi]
    (lo <= min(0, n-m) and hi >= max(0, n-m) assumed); None if no path can."""
    if mode == GLOBAL:
        cands = []
        if hi + 1 <= n:                      # a path can reach diagonal U+1
            cands.append(2 * (hi + 1) - (n - m))
        if lo - 1 >= -m:                     # ... or diagonal L-1
            cands.append((n - m) - 2 * (lo - 1))
        best = None
        for gmin in cands:
            gmax = (m + n - gmin) // 2
            if gmax < 0:
                continue
            g = gmax if sigma_max + 2 * beta >= 0 else 0
            ub = sigma_max * g - 2 * alpha - beta * (m + n - 2 * g - 2)
            best = ub if best is None else max(best, ub)
        return best
    if mode == SEMIGLOBAL:
        def diag_len(d):
            return min(m, n - d) if d >= 0 else min(m + d, n)
        lens = []
        if hi + 1 <= n:
            lens.append(diag_len(hi + 1))
        if lo - 1 >= -m:
            lens.append(diag_len(lo - 1))
        if not lens:
            return None
        return max(sigma_max, 0) * max(lens)
    raise ValueError("band bound defined for global and semi-global only")


def accepts(score_band: int, ub) -> bool:
    return ub is None or score_band >= ub


def accepted_width(q, s, subst, alpha, beta, mode) -> int:
    """Smallest w >= 0 whose banded score passes the acceptance bound.

    S_band(w) never decreases and UB_out(w) never increases with w, so the
    predicate is monotone and bisection finds the smallest accepted w."""
    m, n = len(q), len(s)
    smax = int(max(int(x) for x in __import__("numpy").asarray(subst).ravel()))

    def ok(w):
        return accepts(banded_pair(q, s, subst, alpha, beta, mode, w),
                       ub_outside(m, n, w, smax, alpha, beta, mode))

    lo, hi = 0, max(m, n)
    if ok(0):
        return 0
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return hi


def exact_width(q, s, subst, alpha, beta, mode) -> int:
    """Smallest w whose banded score equals the full score (bisection: the
    banded score is monotone in w and full once the band covers the matrix)."""
    full = align_pair(q, s, subst, alpha, beta, mode)
    lo, hi = -1, max(len(q), len(s))
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if banded_pair(q, s, subst, alpha, beta, mode, mid) == full:
            hi = mid
        else:
            lo = mid
    return hi


# Widest band the banded kernels compute (in diagonals); a pair whose
# accepted band would be wider gets this value as its label.
MAX_BAND = 1024


def band_label(q, s, subst, alpha, beta, mode, max_band: int = MAX_BAND) -> int:
    """Training label of a pair: the smallest accepted half-width w when its
    band (|n - m| + 2w + 1 diagonals) fits in max_band diagonals, else
    max_band (an ordinal 'wider than any band' value)."""
    m, n = len(q), len(s)
    w_cap = (max_band - 1 - abs(n - m)) // 2
    if w_cap < 0:
        return max_band
    wa = accepted_width(q, s, subst, alpha, beta, mode)
    return wa if wa <= w_cap else max_band
