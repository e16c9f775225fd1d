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


# ---- residue-aware bound on band-leaving paths (global mode) ---------------
#
# A study of a tighter certificate than ub_outside; the GPU library does not
# use it.  Loss of a global path: sigma_max*(m+n)/2 - score, a sum of
# non-negative step costs (every diagonal step loses sigma_max - sigma, every
# gap run of L columns alpha - beta + (beta + sigma_max/2)*L, from the gap
# cost alpha + beta*(L-1) of Eq. (4),(5)).  Costs are kept doubled so that
# they stay integers.  Cut Q into seeds of k residues (rows r_s = s*k,
# s < m // k).  A path's node s is its last cell in row r_s, on diagonal d;
# between node s and node s+1 it takes k down-moves and the horizontal moves
# of rows r_s+1 .. r_s+k.  With no gap in between, its k diagonal steps lose
# nothing only if every pair on diagonal d scores sigma_max (the seed matches
# exactly there) and at least delta otherwise (delta: sigma_max minus the next
# lower score); with gaps, a net shift of t > 0 diagonals costs at least one
# run opening plus t gap columns, a shift of t < 0 at least |t| columns (the
# vertical run may have opened earlier), no shift at least an opening plus
# two columns.  The least total over node sequences is a lower bound on
# every path's loss; adding the cost of reaching diagonal e from the nodes on
# either side of the segment where the path first gets there gives a lower
# bound on the loss of every path that visits e.  (Seed matches bounding the
# errors of a region are the q-gram argument used by seed heuristics for
# exact alignment; this is a chaining form of it with the affine costs.)

def _chain_costs(subst, alpha, beta):
    sub = __import__("numpy").asarray(subst, dtype=int)
    smax = int(sub.max())
    lower = sub[sub < smax]
    two_cg = 2 * beta + smax                 # doubled cost of one gap column
    two_a0 = 2 * (alpha - beta)              # doubled cost of opening a run
    two_delta = 2 * (smax - int(lower.max())) if lower.size else None
    pen = two_a0 + 2 * two_cg
    if two_delta is not None:
        pen = min(pen, two_delta)
    return sub, smax, two_cg, two_a0, pen


def seed_chain_visit_bounds(q, s, subst, alpha, beta, k):
    """Doubled lower bounds on the loss of global paths that visit each
    diagonal e (array index e + m, e = -m .. n): (C_up, C_dn, any_fwd,
    any_bwd), C_up valid for e > max(0, n-m) and C_dn for e < min(0, n-m);
    any_fwd (forward chain to the last node plus the tail) and any_bwd
    (backward chain from the first node) bound the loss of every path.
    Needs 0 <= beta <= alpha and k >= 1."""
    import numpy as np
    sub, smax, cg, a0, pen = _chain_costs(subst, alpha, beta)
    q = np.asarray(q, dtype=int)
    s = np.asarray(s, dtype=int)
    m, n = len(q), len(s)
    big = 1 << 60
    d = np.arange(-m, n + 1)
    idx = np.arange(len(d))

    def up(F, a):        # min over j < i of F[j] + a + cg*(i - j)
        x = np.minimum(F + a - cg * idx, big)
        out = np.full(len(F), big, dtype=np.int64)
        out[1:] = np.minimum.accumulate(x[:-1])
        return np.minimum(out + cg * idx, big)

    def dn(F, a):        # min over j > i of F[j] + a + cg*(j - i)
        x = np.minimum(F + a + cg * idx, big)
        out = np.full(len(F), big, dtype=np.int64)
        out[:-1] = np.minimum.accumulate(x[::-1])[::-1][1:]
        return np.minimum(out - cg * idx, big)

    nseed = m // k
    match = np.zeros((nseed, len(d)), dtype=bool)
    for si in range(nseed if n else 0):
        r = si * k
        ok = (r + d >= 0) & (r + d + k <= n)
        good = ok.copy()
        for t in range(k):
            col = np.where(ok, r + d + t, 0)
            good &= sub[q[r + t], s[col]] == smax
        match[si] = good

    def seg(F, si, a_up, a_dn):
        stay = np.minimum(F + np.where(match[si], 0, pen), big)
        return np.minimum(stay, np.minimum(up(F, a_up), dn(F, a_dn)))

    F = [np.where(d == 0, 0, np.where(d > 0, a0 + cg * d, big)).astype(np.int64)]
    for si in range(nseed):
        F.append(seg(F[-1], si, a0, 0))
    e = n - m
    B = [None] * (nseed + 1)
    B[nseed] = np.where(d == e, 0, np.where(d < e, a0 + cg * (e - d), cg * (d - e))).astype(np.int64)
    for si in range(nseed - 1, -1, -1):
        # from node diagonal x: up to x' > x costs a0 + cg*(x'-x), down cg*(x-x')
        B[si] = seg(B[si + 1], si, 0, a0)

    c_up = np.full(len(d), big, dtype=np.int64)
    c_dn = np.full(len(d), big, dtype=np.int64)
    for si in range(nseed + 1):
        Fs = F[si]
        reach_up = np.minimum(Fs, up(Fs, a0))       # at diagonal e going up
        reach_dn = np.minimum(Fs, dn(Fs, 0))        # at diagonal e going down
        if si == nseed:
            back_dn = np.where(d >= e, cg * (d - e), big)
            back_up = np.where(d <= e, np.where(d < e, a0, 0) + cg * (e - d), big)
        else:
            Bn = B[si + 1]
            back_dn = np.minimum(Bn, np.minimum(up(Bn, 0), dn(Bn, 0)))
            back_up = np.minimum(Bn, np.minimum(dn(Bn, a0), up(Bn, 0)))
        c_up = np.minimum(c_up, np.minimum(reach_up + back_dn, big))
        c_dn = np.minimum(c_dn, np.minimum(reach_dn + back_up, big))
    # a path that visits e beyond the band also visits every diagonal between
    lo0, hi0 = min(0, n - m), max(0, n - m)
    top = idx[d > hi0]
    if len(top):
        c_up[top] = np.maximum.accumulate(c_up[top])
    bot = idx[d < lo0][::-1]
    if len(bot):
        c_dn[bot] = np.maximum.accumulate(c_dn[bot])
    any_fwd = int(np.min(np.minimum(F[nseed] + B[nseed], big)))
    any_bwd = int(B[0][m])
    return c_up, c_dn, any_fwd, any_bwd


def seed_chain_ub_outside(q, s, subst, alpha, beta, k, lo, hi, bounds=None):
    """Upper bound on the score of every global path that visits a diagonal
    outside [lo, hi] (lo <= min(0, n-m), hi >= max(0, n-m)), from the seed
    chain; None if no path can leave.  `bounds` reuses a result of
    seed_chain_visit_bounds for the same pair."""
    m, n = len(q), len(s)
    c_up, c_dn = (bounds if bounds is not None else seed_chain_visit_bounds(q, s, subst, alpha, beta, k))[:2]
    cands = []
    if hi + 1 <= n:
        cands.append(int(c_up[hi + 1 + m]))
    if lo - 1 >= -m:
        cands.append(int(c_dn[lo - 1 + m]))
    if not cands:
        return None
    smax = int(__import__("numpy").asarray(subst).max())
    return (smax * (m + n) - min(cands)) // 2


def seed_chain_accepted_width(q, s, subst, alpha, beta, k) -> int:
    """Smallest w >= 0 whose banded global score passes the smaller of the
    closed-form bound and the seed-chain bound (both are sound, so either
    accepts only exact scores)."""
    import numpy as np
    m, n = len(q), len(s)
    smax = int(np.asarray(subst).max())
    bounds = seed_chain_visit_bounds(q, s, subst, alpha, beta, k)

    def ok(w):
        lo, hi = band_limits(m, n, w)
        ub1 = ub_outside(m, n, w, smax, alpha, beta, GLOBAL)
        ub2 = seed_chain_ub_outside(q, s, subst, alpha, beta, k, lo, hi, bounds)
        ub = ub1 if ub2 is None else (ub2 if ub1 is None else min(ub1, ub2))
        return accepts(banded_pair(q, s, subst, alpha, beta, GLOBAL, w), ub)

    if ok(0):
        return 0
    lo_w, hi_w = 0, max(m, n)
    while hi_w - lo_w > 1:
        mid = (lo_w + hi_w) // 2
        if ok(mid):
            hi_w = mid
        else:
            lo_w = mid
    return hi_w
