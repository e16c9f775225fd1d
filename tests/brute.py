"""Brute-force alignment enumeration for tiny pairs (test infrastructure).

Independent of any dynamic program: every alignment of two sequences is
enumerated as a string of moves (D = q_i aligned to s_j, V = q_i against a
gap, H = s_j against a gap) and scored by its definition -- the sum of sigma
over aligned columns minus alpha + (k-1)*beta for every maximal run of k gap
columns of the same kind (paper Eq. (4),(5) state that cost per gap).

Modes, by their definitions in section 2.1 of the paper:
* global: best alignment of the whole of both sequences;
* local: best alignment of any substring of Q with any substring of S, the
  empty alignment (score 0) included;
* semi-global: gaps before the first and after the last aligned residue are
  free, i.e. the best global alignment of Q[a:c] with S[b:d] where the part
  cut off at the start is a prefix of only one sequence (a == 0 or b == 0)
  and likewise at the end (c == m or d == n).
An optional `cell_ok(i, j)` restricts the paths to allowed DP cells, which
gives band-restricted and band-leaving scores.
"""
from __future__ import annotations

NEG = float("-inf")


def _global_paths(q, s, subst, alpha, beta, i0, j0, cell_ok=None, escape=False):
    """Max over all move strings from (i0, j0) to (len(q)+i0, len(s)+j0) in
    absolute cell coordinates.  With escape=False every visited cell must
    satisfy cell_ok; with escape=True only paths that visit at least one cell
    failing cell_ok count."""
    m, n = len(q), len(s)
    best = NEG

    def rec(i, j, last, score, out):
        nonlocal best
        if cell_ok is not None and not cell_ok(i + i0, j + j0):
            if not escape:
                return
            out = True
        if i == m and j == n:
            if score > best and (out or not escape):
                best = score
            return
        if i < m and j < n:
            rec(i + 1, j + 1, "D", score + int(subst[q[i]][s[j]]), out)
        if i < m:
            rec(i + 1, j, "V", score - (beta if last == "V" else alpha), out)
        if j < n:
            rec(i, j + 1, "H", score - (beta if last == "H" else alpha), out)

    rec(0, 0, None, 0, False)
    return best


def global_score(q, s, subst, alpha, beta, cell_ok=None, escape=False):
    return _global_paths(q, s, subst, alpha, beta, 0, 0, cell_ok, escape)


def local_score(q, s, subst, alpha, beta, cell_ok=None):
    m, n = len(q), len(s)
    best = NEG
    for a in range(m + 1):
        for c in range(a, m + 1):
            for b in range(n + 1):
                for d in range(b, n + 1):
                    v = _global_paths(q[a:c], s[b:d], subst, alpha, beta, a, b, cell_ok)
                    best = max(best, v)
    return best


def semiglobal_score(q, s, subst, alpha, beta, cell_ok=None, escape=False):
    m, n = len(q), len(s)
    best = NEG
    for a in range(m + 1):
        for b in range(n + 1):
            if a != 0 and b != 0:
                continue
            for c in range(a, m + 1):
                for d in range(b, n + 1):
                    if c != m and d != n:
                        continue
                    v = _global_paths(q[a:c], s[b:d], subst, alpha, beta, a, b, cell_ok, escape)
                    best = max(best, v)
    return best


SCORERS = {0: global_score, 1: semiglobal_score, 2: local_score}


def all_alignments(q, s, subst, alpha, beta):
    """Every global alignment of q against s as (columns, score): columns is
    a string over 'M' (q_i with s_j), 'I' (q_i against a gap), 'D' (s_j
    against a gap); the score is computed by the definition above, column
    by column."""
    m, n = len(q), len(s)
    out = []

    def rec(i, j, last, score, cols):
        if i == m and j == n:
            out.append(("".join(cols), score))
            return
        if i < m and j < n:
            cols.append("M")
            rec(i + 1, j + 1, "M", score + int(subst[q[i]][s[j]]), cols)
            cols.pop()
        if i < m:
            cols.append("I")
            rec(i + 1, j, "I", score - (beta if last == "I" else alpha), cols)
            cols.pop()
        if j < n:
            cols.append("D")
            rec(i, j + 1, "D", score - (beta if last == "D" else alpha), cols)
            cols.pop()

    rec(0, 0, None, 0, [])
    return out
