"""CPU oracle for score-only pairwise alignment -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports, links
or calls it, and the two share no code (no kernels, headers, helpers, tables
or pre-/post-processing).  The only code both sides receive is the seeded
input generator module, which holds none of the method's arithmetic.

What it computes is the plain definition of the optimal alignment score
(paper section 2.1, Eq. (1)-(5) and the local / global / semi-global mode
paragraphs), written in ``oracle.c`` as a textbook row-by-row dynamic program
in 64-bit integers.  ``band.py`` holds the banded score's acceptance bound,
the band label and a residue-aware (seed-chain) bound on band-leaving paths, ``mlp.py`` the band network in float64, ``features.py``
the per-pair k-mer features.  How each function is pinned to something other
than itself is stated in the function's docstring and in the tests under
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

GLOBAL, SEMIGLOBAL, LOCAL = 0, 1, 2
MODES = {"global": GLOBAL, "semiglobal": SEMIGLOBAL, "local": LOCAL}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the C oracle with gcc (plain -O2, no vector intrinsics)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-pthread",
                           _SRC, "-o", tmp])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, i32, p = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.oracle_align_pair.restype = i64
    lib.oracle_align_pair.argtypes = [p, i64, p, i64, p, i32, i64, i64, i32]
    lib.oracle_banded_pair.restype = i64
    lib.oracle_banded_pair.argtypes = [p, i64, p, i64, p, i32, i64, i64, i32, i64]
    lib.oracle_align_batch.restype = None
    lib.oracle_align_batch.argtypes = [p, p, p, p, i64, p, i32, i64, i64, i32, i32, p]
    lib.oracle_diag_band_pair.restype = i64
    lib.oracle_diag_band_pair.argtypes = [p, i64, p, i64, p, i32, i64, i64, i32, i64, i64]
    lib.oracle_diag_band_batch.restype = None
    lib.oracle_diag_band_batch.argtypes = [p, p, p, p, i64, p, i32, i64, i64, i32, p, p, i32, p]
    lib.oracle_banded_batch.restype = None
    lib.oracle_banded_batch.argtypes = [p, p, p, p, i64, p, i32, i64, i64, i32, p, i32, p]
    lib.oracle_alignment_score.restype = i64
    lib.oracle_alignment_score.argtypes = [p, i64, p, i64, p, i32, i64, i64, i32, p, i64, p]
    lib.oracle_traceback_pair.restype = i64
    lib.oracle_traceback_pair.argtypes = [p, i64, p, i64, p, i32, i64, i64, i32, p, p]
    lib.oracle_traceback_batch.restype = None
    lib.oracle_traceback_batch.argtypes = [p, p, p, p, i64, p, i32, i64, i64, i32, i32, p, p, p]
    lib.oracle_alignment_score_batch.restype = None
    lib.oracle_alignment_score_batch.argtypes = [p, p, p, p, i64, p, i32, i64, i64, i32, i32, p, p, p]
    _lib = lib
    return lib


def _u8(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint8))


def _subst(subst) -> tuple[np.ndarray, int]:
    s = np.ascontiguousarray(np.asarray(subst, dtype=np.int8))
    asz = s.shape[0]
    assert s.shape == (asz, asz)
    return s, asz


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return len(os.sched_getaffinity(0))


def align_pair(q, s, subst, alpha: int, beta: int, mode: int) -> int:
    """Optimal score of one pair (codes 0..asz-1), full dynamic program."""
    q, s = _u8(q), _u8(s)
    sub, asz = _subst(subst)
    return int(_load().oracle_align_pair(_ptr(q), len(q), _ptr(s), len(s), _ptr(sub), asz,
                                          int(alpha), int(beta), int(mode)))


def banded_pair(q, s, subst, alpha: int, beta: int, mode: int, w: int) -> int:
    """Score restricted to diagonals min(0,n-m)-w <= j-i <= max(0,n-m)+w."""
    q, s = _u8(q), _u8(s)
    sub, asz = _subst(subst)
    return int(_load().oracle_banded_pair(_ptr(q), len(q), _ptr(s), len(s), _ptr(sub), asz,
                                           int(alpha), int(beta), int(mode), int(w)))


def align_batch(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                nthreads: int | None = None) -> np.ndarray:
    """Scores of every pair p: A[offs_a[p]:offs_a[p+1]] vs B[offs_b[p]:offs_b[p+1]]."""
    sa, sb = _u8(seqs_a), _u8(seqs_b)
    oa = np.ascontiguousarray(offs_a, dtype=np.int64)
    ob = np.ascontiguousarray(offs_b, dtype=np.int64)
    n = len(oa) - 1
    assert len(ob) == n + 1
    sub, asz = _subst(subst)
    out = np.zeros(n, dtype=np.int64)
    _load().oracle_align_batch(_ptr(sa), _ptr(oa), _ptr(sb), _ptr(ob), n, _ptr(sub), asz,
                               int(alpha), int(beta), int(mode),
                               nthreads or default_threads(), _ptr(out))
    return out


def banded_batch(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                 band_w, nthreads: int | None = None) -> np.ndarray:
    """Banded scores of every pair, half-width band_w[p] for pair p."""
    sa, sb = _u8(seqs_a), _u8(seqs_b)
    oa = np.ascontiguousarray(offs_a, dtype=np.int64)
    ob = np.ascontiguousarray(offs_b, dtype=np.int64)
    n = len(oa) - 1
    w = np.ascontiguousarray(band_w, dtype=np.int64)
    assert len(w) == n
    sub, asz = _subst(subst)
    out = np.zeros(n, dtype=np.int64)
    _load().oracle_banded_batch(_ptr(sa), _ptr(oa), _ptr(sb), _ptr(ob), n, _ptr(sub), asz,
                                int(alpha), int(beta), int(mode), _ptr(w),
                                nthreads or default_threads(), _ptr(out))
    return out


def diag_band_pair(q, s, subst, alpha: int, beta: int, mode: int, lo: int, hi: int) -> int:
    """Score restricted to diagonals lo <= j-i <= hi (boundary cells included)."""
    q, s = _u8(q), _u8(s)
    sub, asz = _subst(subst)
    return int(_load().oracle_diag_band_pair(_ptr(q), len(q), _ptr(s), len(s), _ptr(sub), asz,
                                              int(alpha), int(beta), int(mode), int(lo), int(hi)))


def diag_band_batch(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                    lo, hi, nthreads: int | None = None) -> np.ndarray:
    """Scores of every pair restricted to its own diagonal limits lo[p] <= j-i <= hi[p]."""
    sa, sb = _u8(seqs_a), _u8(seqs_b)
    oa = np.ascontiguousarray(offs_a, dtype=np.int64)
    ob = np.ascontiguousarray(offs_b, dtype=np.int64)
    n = len(oa) - 1
    lo = np.ascontiguousarray(lo, dtype=np.int64)
    hi = np.ascontiguousarray(hi, dtype=np.int64)
    sub, asz = _subst(subst)
    out = np.zeros(n, dtype=np.int64)
    _load().oracle_diag_band_batch(_ptr(sa), _ptr(oa), _ptr(sb), _ptr(ob), n, _ptr(sub), asz,
                                   int(alpha), int(beta), int(mode), _ptr(lo), _ptr(hi),
                                   nthreads or default_threads(), _ptr(out))
    return out


# ---- alignments (the "Traceback" paragraph of the paper's section 2.1) ----

INVALID = -(1 << 63)   # oracle_alignment_score's value for an alignment the mode does not admit


def alignment_score(q, s, subst, alpha: int, beta: int, mode: int, ops, span) -> int:
    """Score of one alignment by its definition (sigma over aligned columns,
    alpha + (k-1) beta per maximal gap run), or INVALID when its columns
    ('M', 'I' = q_i against a gap, 'D' = s_j against a gap) do not consume
    exactly span = (a0, a1, b0, b1) or the mode does not admit that span."""
    q, s = _u8(q), _u8(s)
    sub, asz = _subst(subst)
    o = np.frombuffer(ops.encode() if isinstance(ops, str) else bytes(ops), dtype=np.uint8).copy()
    sp = np.ascontiguousarray(span, dtype=np.int32)
    return int(_load().oracle_alignment_score(_ptr(q), len(q), _ptr(s), len(s), _ptr(sub), asz,
                                              int(alpha), int(beta), int(mode),
                                              _ptr(o) if len(o) else _ptr(np.zeros(1, np.uint8)),
                                              len(o), _ptr(sp)))


def traceback_pair(q, s, subst, alpha: int, beta: int, mode: int):
    """(score, ops string, span (a0, a1, b0, b1)) of one optimal alignment."""
    q, s = _u8(q), _u8(s)
    sub, asz = _subst(subst)
    ops = np.zeros(len(q) + len(s) + 1, dtype=np.uint8)
    sp = np.zeros(5, dtype=np.int32)
    sc = int(_load().oracle_traceback_pair(_ptr(q), len(q), _ptr(s), len(s), _ptr(sub), asz,
                                           int(alpha), int(beta), int(mode), _ptr(ops), _ptr(sp)))
    return sc, ops[:sp[0]].tobytes().decode(), tuple(int(x) for x in sp[1:])


def alignment_score_batch(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                          ops, span, nthreads: int | None = None) -> np.ndarray:
    """Score of every pair's alignment (INVALID where it is not one): pair p's
    columns are ops[(offs_a[p] - offs_a[0]) + (offs_b[p] - offs_b[0]):][:span[p][0]],
    span[p] = (n_ops, a0, a1, b0, b1)."""
    sa, sb = _u8(seqs_a), _u8(seqs_b)
    oa = np.ascontiguousarray(offs_a, dtype=np.int64)
    ob = np.ascontiguousarray(offs_b, dtype=np.int64)
    n = len(oa) - 1
    o = np.ascontiguousarray(ops, dtype=np.uint8)
    sp = np.ascontiguousarray(span, dtype=np.int32).reshape(n, 5)
    sub, asz = _subst(subst)
    out = np.zeros(n, dtype=np.int64)
    _load().oracle_alignment_score_batch(_ptr(sa), _ptr(oa), _ptr(sb), _ptr(ob), n, _ptr(sub), asz,
                                         int(alpha), int(beta), int(mode),
                                         nthreads or default_threads(), _ptr(o), _ptr(sp), _ptr(out))
    return out


def traceback_batch(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                    nthreads: int | None = None):
    """(scores, ops, span) of every pair, in the layout of alignment_score_batch."""
    sa, sb = _u8(seqs_a), _u8(seqs_b)
    oa = np.ascontiguousarray(offs_a, dtype=np.int64)
    ob = np.ascontiguousarray(offs_b, dtype=np.int64)
    n = len(oa) - 1
    sub, asz = _subst(subst)
    ops = np.zeros(max(1, int(oa[-1] - oa[0] + ob[-1] - ob[0])), dtype=np.uint8)
    sp = np.zeros((n, 5), dtype=np.int32)
    out = np.zeros(n, dtype=np.int64)
    _load().oracle_traceback_batch(_ptr(sa), _ptr(oa), _ptr(sb), _ptr(ob), n, _ptr(sub), asz,
                                   int(alpha), int(beta), int(mode), nthreads or default_threads(),
                                   _ptr(ops), _ptr(sp), _ptr(out))
    return out, ops, sp
