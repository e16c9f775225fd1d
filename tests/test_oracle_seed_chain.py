"""Pins of the oracle's seed-chain bound on band-leaving global paths
(oracle/band.py: seed_chain_visit_bounds, seed_chain_ub_outside,
seed_chain_accepted_width), a residue-aware alternative to the closed-form
acceptance bound that the GPU library does not use.

* Soundness: the chain's bound on the loss of every path is at most the
  optimal loss (full dynamic program) on random pairs, including scorings
  where an indel pair costs less than a mismatch; and on random small pairs (several alphabets, scores of either
  sign, related and unrelated pairs, seed lengths 1..5) the bound is at least
  the exact best score of the paths that leave the band, which an
  independent two-layer dynamic program below computes; that program is
  itself pinned to brute-force enumeration of every alignment.
* Tightness: on pairs of the 1-5 kb workload's law the widths it accepts
  cover at most 0.6 of the cells the closed form's widths cover, and every
  width it accepts gives the full score.
"""
import numpy as np
import pytest

import brute
from oracle import GLOBAL, band

NEG = float("-inf")


def _leave_best(q, s, sub, alpha, beta, lo, hi):
    """Best global score over paths that visit a cell with j - i outside
    [lo, hi]: Gotoh's recurrences (Eq. (1),(4),(5)) with a second layer for
    paths that have left."""
    m, n = len(q), len(s)

    def out(i, j):
        return not (lo <= j - i <= hi)

    H = [[[NEG, NEG] for _ in range(n + 1)] for _ in range(m + 1)]
    E = [[[NEG, NEG] for _ in range(n + 1)] for _ in range(m + 1)]
    F = [[[NEG, NEG] for _ in range(n + 1)] for _ in range(m + 1)]
    H[0][0][1 if out(0, 0) else 0] = 0
    for i in range(m + 1):
        for j in range(n + 1):
            if i == 0 and j == 0:
                continue
            o = out(i, j)
            for f in (0, 1):
                t = 1 if (f or o) else 0
                if j > 0:
                    v = max(H[i][j - 1][f] - alpha, E[i][j - 1][f] - beta)
                    E[i][j][t] = max(E[i][j][t], v)
                if i > 0:
                    v = max(H[i - 1][j][f] - alpha, F[i - 1][j][f] - beta)
                    F[i][j][t] = max(F[i][j][t], v)
                if i > 0 and j > 0:
                    H[i][j][t] = max(H[i][j][t], H[i - 1][j - 1][f] + int(sub[q[i - 1]][s[j - 1]]))
            for t in (0, 1):
                H[i][j][t] = max(H[i][j][t], E[i][j][t], F[i][j][t])
    return H[m][n][1]


def _scoring(rng, asz):
    sub = rng.integers(-4, 5, size=(asz, asz))
    if rng.random() < 0.5:
        sub = np.full((asz, asz), int(rng.integers(-4, 0)))
        np.fill_diagonal(sub, int(rng.integers(1, 5)))
    beta = int(rng.integers(0, 4))
    alpha = beta + int(rng.integers(0, 5))
    return sub, alpha, beta


def _pair(rng, asz, max_len):
    m = int(rng.integers(0, max_len + 1))
    q = rng.integers(0, asz, size=m).tolist()
    if m and rng.random() < 0.6:          # a related pair: edits of q
        s = list(q)
        for _ in range(int(rng.integers(0, 4))):
            op = rng.integers(0, 3)
            pos = int(rng.integers(0, len(s) + 1))
            if op == 0 and pos < len(s):
                s[pos] = int(rng.integers(0, asz))
            elif op == 1:
                s.insert(pos, int(rng.integers(0, asz)))
            elif pos < len(s):
                del s[pos]
    else:
        s = rng.integers(0, asz, size=int(rng.integers(0, max_len + 1))).tolist()
    return q, s


def test_leave_dp_matches_enumeration():
    rng = np.random.default_rng(4100)
    checked = 0
    for _ in range(60):
        sub, alpha, beta = _scoring(rng, 3)
        q, s = _pair(rng, 3, 6)
        m, n = len(q), len(s)
        for w in range(0, max(m, n) + 1):
            lo, hi = band.band_limits(m, n, w)
            want = brute.global_score(q, s, sub, alpha, beta,
                                      cell_ok=lambda i, j: lo <= j - i <= hi, escape=True)
            assert _leave_best(q, s, sub, alpha, beta, lo, hi) == want, (q, s, w)
            checked += 1
    assert checked > 150


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_seed_chain_bound_sound(oracle_mod, k):
    rng = np.random.default_rng(4110 + k)
    checked = 0
    for _ in range(45):
        asz = int(rng.integers(2, 5))
        sub, alpha, beta = _scoring(rng, asz)
        q, s = _pair(rng, asz, 16)
        m, n = len(q), len(s)
        bounds = band.seed_chain_visit_bounds(q, s, sub, alpha, beta, k)
        full = oracle_mod.align_pair(q, s, sub, alpha, beta, GLOBAL)
        lo0, hi0 = min(0, n - m), max(0, n - m)
        limits = [band.band_limits(m, n, w) for w in range(0, max(m, n) + 1, 2)]
        limits += [(lo0 - int(rng.integers(0, 4)), hi0 + int(rng.integers(0, 4))) for _ in range(2)]
        for lo, hi in limits:
            ub = band.seed_chain_ub_outside(q, s, sub, alpha, beta, k, lo, hi, bounds)
            best = _leave_best(q, s, sub, alpha, beta, lo, hi)
            if ub is None:
                assert best == NEG, (q, s, lo, hi)
                continue
            assert best <= ub, (k, q, s, sub.tolist(), alpha, beta, lo, hi, best, ub)
            checked += 1
            sb = oracle_mod.diag_band_pair(q, s, sub, alpha, beta, GLOBAL, lo, hi)
            if sb >= ub:
                assert sb == full
    assert checked > 150


def test_seed_chain_narrower_than_closed_form(oracle_mod):
    """Widths accepted with seed length 4 on 1-2 kb pairs of the 1-5 kb
    workload's law (divergence up to 10%, half indels; match 2, mismatch
    -3, alpha 5, beta 2) cover at most 0.6 of the band cells of the
    closed form's widths; each accepted band gives the full score."""
    from paper_2205_07610_amd import synth
    b = synth.config4_like(8, 4120, min_len=1000, max_len=2000)
    cells_cf = cells_chain = 0
    for p in range(8):
        q = b.seqs_a[b.offs_a[p]:b.offs_a[p + 1]]
        s = b.seqs_b[b.offs_b[p]:b.offs_b[p + 1]]
        m, n = len(q), len(s)
        w_cf = band.accepted_width(q, s, b.subst, b.alpha, b.beta, GLOBAL)
        w_ch = band.seed_chain_accepted_width(q, s, b.subst, b.alpha, b.beta, 4)
        assert w_ch <= w_cf
        assert (oracle_mod.banded_pair(q, s, b.subst, b.alpha, b.beta, GLOBAL, w_ch)
                == oracle_mod.align_pair(q, s, b.subst, b.alpha, b.beta, GLOBAL))
        cells_cf += m * (abs(n - m) + 2 * w_cf + 1)
        cells_chain += m * (abs(n - m) + 2 * w_ch + 1)
    assert cells_chain <= 0.6 * cells_cf, (cells_chain, cells_cf)


def _cheap_gap_scoring(rng, asz):
    sub = np.full((asz, asz), -int(rng.integers(3, 6)))
    np.fill_diagonal(sub, int(rng.integers(1, 5)))
    beta = int(rng.integers(0, 2))
    return sub, beta + int(rng.integers(0, 2)), beta


@pytest.mark.parametrize("k", [1, 2, 3, 4, 7])
def test_seed_chain_any_path_bound(oracle_mod, k):
    """Forward and backward chain values never exceed twice the optimal
    loss sigma_max*(m+n)/2 - score, for ordinary and cheap-gap scorings."""
    rng = np.random.default_rng(4130 + k)
    for it in range(120):
        asz = int(rng.integers(2, 5))
        sub, alpha, beta = (_cheap_gap_scoring if it % 2 else _scoring)(rng, asz)
        q, s = _pair(rng, asz, 60)
        m, n = len(q), len(s)
        full = oracle_mod.align_pair(q, s, sub, alpha, beta, GLOBAL)
        loss2 = int(sub.max()) * (m + n) - 2 * full
        _, _, fwd, bwd = band.seed_chain_visit_bounds(q, s, sub, alpha, beta, k)
        assert fwd <= loss2 and bwd <= loss2, (k, q, s, sub.tolist(), alpha, beta, fwd, bwd, loss2)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_seed_chain_bound_sound_cheap_gaps(oracle_mod, k):
    """Leaving paths under scorings whose indel pairs undercut a mismatch,
    and bands one or two diagonals wide, where the best leaving path goes
    well past the band."""
    rng = np.random.default_rng(4140 + k)
    checked = 0
    for _ in range(40):
        asz = int(rng.integers(2, 5))
        sub, alpha, beta = _cheap_gap_scoring(rng, asz)
        q, s = _pair(rng, asz, 14)
        m, n = len(q), len(s)
        bounds = band.seed_chain_visit_bounds(q, s, sub, alpha, beta, k)
        for w in range(0, 3):
            lo, hi = band.band_limits(m, n, w)
            ub = band.seed_chain_ub_outside(q, s, sub, alpha, beta, k, lo, hi, bounds)
            best = _leave_best(q, s, sub, alpha, beta, lo, hi)
            if ub is None:
                assert best == NEG
                continue
            assert best <= ub, (k, q, s, sub.tolist(), alpha, beta, lo, hi, best, ub)
            checked += 1
    assert checked > 60


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_seed_chain_each_side_each_diagonal(oracle_mod, k):
    """C_up(e) and C_dn(e), one side at a time, at every diagonal past the
    corner diagonals: never above twice the least loss of the paths that
    visit e (upper side: paths reaching j - i >= e; lower: j - i <= e)."""
    rng = np.random.default_rng(4150 + k)
    checked = 0
    for it in range(50):
        asz = int(rng.integers(2, 5))
        sub, alpha, beta = (_cheap_gap_scoring if it % 3 == 0 else _scoring)(rng, asz)
        q, s = _pair(rng, asz, 12)
        m, n = len(q), len(s)
        smax = int(sub.max())
        c_up, c_dn, _, _ = band.seed_chain_visit_bounds(q, s, sub, alpha, beta, k)
        for e in range(max(0, n - m) + 1, n + 1):
            best = _leave_best(q, s, sub, alpha, beta, -m - 1, e - 1)
            assert c_up[e + m] <= smax * (m + n) - 2 * best, ("up", k, q, s, e)
            checked += 1
        for e in range(-m, min(0, n - m)):
            best = _leave_best(q, s, sub, alpha, beta, e + 1, n + 1)
            assert c_dn[e + m] <= smax * (m + n) - 2 * best, ("down", k, q, s, e)
            checked += 1
    assert checked > 300
