"""Seeded synthetic inputs for the five workloads (no alignment arithmetic here).

This module is the only code that both the GPU path's callers and the CPU
oracle's callers share.  It draws residues, lengths and mutations and builds
substitution matrices; it computes no alignment score, bound or feature.

The paper's own data (Mason-simulated Illumina reads and PBSIM PacBio reads
from GRCh38 chr10, section 4.1) is not available, so every workload is drawn
from the recipes below, with the shapes of the paper's short-read, mixed-length
and long-read experiments:

* residues: uniform codes 0..3 (DNA, A C G T) or 0..19 (protein);
* mutation model, applied per source residue: substitution (a uniformly
  different residue) with p_sub, an insertion of L ~ Geometric(1/2) random
  residues before it with p_ins, a deletion of L ~ Geometric(1/2) residues
  starting at it with p_del (geometric lengths have mean 2);
* "divergence d, half indels" means p_sub = d/2, p_ins = p_del = d/4.

All penalties are magnitudes: a gap of length k costs alpha + (k-1)*beta
(paper Eq. (4),(5)); "gap open -5, extend -2" is alpha = 5, beta = 2.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "synth_gen.c")
_GEN_LIB = os.path.join(_HERE, "libsynth_gen.so")
_gen = None


def build_generator() -> str:
    """Compile the multithreaded C generator (plain gcc -O2)."""
    tmp = _GEN_LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-pthread",
                           _GEN_SRC, "-o", tmp])
    os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _generator():
    global _gen
    if _gen is None:
        if not os.path.exists(_GEN_LIB) or os.path.getmtime(_GEN_LIB) < os.path.getmtime(_GEN_SRC):
            build_generator()
        L = ctypes.CDLL(_GEN_LIB)
        p, i64, u64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        L.synth_residues.restype = None
        L.synth_residues.argtypes = [u64, i64, p, i32, p, i32]
        L.synth_mutate.restype = None
        L.synth_mutate.argtypes = [u64, i64, p, p, p, p, p, i32, p, p, p, i32]
        _gen = L
    return _gen


def _threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def native_csr(seed: int, lens, asz: int, nthreads: int | None = None):
    """Uniform residues for sequences of the given lengths (C generator)."""
    lens = np.asarray(lens, dtype=np.int64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    out = np.empty(int(offs[-1]), dtype=np.uint8)
    _generator().synth_residues(int(seed), len(lens), _ptr(offs), int(asz), _ptr(out),
                                nthreads or _threads())
    return out, offs


def native_mutate(seed: int, seqs, offs, p_sub, p_ins, p_del, asz: int,
                  nthreads: int | None = None):
    """The mutation model of `mutate`, drawn by the C generator (two passes:
    lengths, then residues, from the same per-sequence streams)."""
    seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    n = len(offs) - 1
    ps, pi, pd = (np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), (n,)))
                  for v in (p_sub, p_ins, p_del))
    lens = np.zeros(n, dtype=np.int64)
    g = _generator()
    nt = nthreads or _threads()
    g.synth_mutate(int(seed), n, _ptr(offs), _ptr(seqs), _ptr(ps), _ptr(pi), _ptr(pd), int(asz),
                   None, None, _ptr(lens), nt)
    new_offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=new_offs[1:])
    out = np.empty(int(new_offs[-1]), dtype=np.uint8)
    g.synth_mutate(int(seed), n, _ptr(offs), _ptr(seqs), _ptr(ps), _ptr(pi), _ptr(pd), int(asz),
                   _ptr(new_offs), _ptr(out), None, nt)
    return out, new_offs

MODE_GLOBAL, MODE_SEMIGLOBAL, MODE_LOCAL = 0, 1, 2


@dataclasses.dataclass
class Batch:
    """A batch of pairs in CSR form: pair p is A[offs_a[p]:offs_a[p+1]] vs B[...]."""
    name: str
    seqs_a: np.ndarray   # uint8 codes
    offs_a: np.ndarray   # int64 [n_pairs + 1]
    seqs_b: np.ndarray
    offs_b: np.ndarray
    subst: np.ndarray    # int8 [asz, asz], subst[q, s] = sigma(q, s)
    alpha: int           # cost of a gap's first residue
    beta: int            # cost of each further residue of the gap
    mode: int            # 0 global, 1 semi-global, 2 local

    @property
    def n_pairs(self) -> int:
        return len(self.offs_a) - 1

    @property
    def lens_a(self) -> np.ndarray:
        return np.diff(self.offs_a)

    @property
    def lens_b(self) -> np.ndarray:
        return np.diff(self.offs_b)

    def cells(self) -> int:
        return int(np.sum(self.lens_a.astype(np.int64) * self.lens_b.astype(np.int64)))

    def subset(self, idx) -> "Batch":
        """Pairs idx (in that order) as a new, compact batch."""
        idx = np.asarray(idx, dtype=np.int64)
        sa, oa = _gather(self.seqs_a, self.offs_a, idx)
        sb, ob = _gather(self.seqs_b, self.offs_b, idx)
        return Batch(self.name, sa, oa, sb, ob, self.subst, self.alpha, self.beta, self.mode)

    def pair(self, p: int) -> tuple[np.ndarray, np.ndarray]:
        return (self.seqs_a[self.offs_a[p]:self.offs_a[p + 1]],
                self.seqs_b[self.offs_b[p]:self.offs_b[p + 1]])


def _gather(seqs, offs, idx):
    lens = (offs[idx + 1] - offs[idx]).astype(np.int64)
    new_offs = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(lens, out=new_offs[1:])
    total = int(new_offs[-1])
    if total == 0:
        return np.zeros(0, dtype=np.uint8), new_offs
    starts = np.repeat(offs[idx] - new_offs[:-1], lens)
    return seqs[np.arange(total, dtype=np.int64) + starts], new_offs


def from_pairs(name, pairs, subst, alpha, beta, mode) -> Batch:
    """Build a batch from a list of (a, b) code arrays."""
    la = np.array([len(a) for a, _ in pairs], dtype=np.int64)
    lb = np.array([len(b) for _, b in pairs], dtype=np.int64)
    oa = np.zeros(len(pairs) + 1, dtype=np.int64)
    ob = np.zeros(len(pairs) + 1, dtype=np.int64)
    np.cumsum(la, out=oa[1:])
    np.cumsum(lb, out=ob[1:])
    sa = (np.concatenate([np.asarray(a, dtype=np.uint8) for a, _ in pairs])
          if int(oa[-1]) else np.zeros(0, np.uint8))
    sb = (np.concatenate([np.asarray(b, dtype=np.uint8) for _, b in pairs])
          if int(ob[-1]) else np.zeros(0, np.uint8))
    return Batch(name, sa, oa, sb, ob, np.asarray(subst, dtype=np.int8), int(alpha), int(beta),
                 int(mode))


# ---------------------------------------------------------------- scoring ----

def dna_subst(match: int = 2, mismatch: int = -3) -> np.ndarray:
    s = np.full((4, 4), mismatch, dtype=np.int8)
    np.fill_diagonal(s, match)
    return s


def protein_subst(rng: np.random.Generator) -> np.ndarray:
    """Symmetric 20x20 int8: diagonal U[4,11], off-diagonal U[-4,3]."""
    s = np.zeros((20, 20), dtype=np.int8)
    iu = np.triu_indices(20, 1)
    off = rng.integers(-4, 4, size=len(iu[0]))
    s[iu] = off
    s[(iu[1], iu[0])] = off
    np.fill_diagonal(s, rng.integers(4, 12, size=20))
    return s


# --------------------------------------------------------------- residues ----

def random_csr(rng: np.random.Generator, lens, asz: int):
    lens = np.asarray(lens, dtype=np.int64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    return rng.integers(0, asz, size=int(offs[-1]), dtype=np.uint8), offs


def mutate(rng: np.random.Generator, seqs, offs, p_sub, p_ins, p_del, asz: int):
    """Apply the per-residue mutation model to every sequence of a CSR batch.

    p_sub / p_ins / p_del are scalars or per-sequence arrays.  Deletions never
    run past the end of their own sequence.
    """
    seqs = np.asarray(seqs, dtype=np.uint8)
    offs = np.asarray(offs, dtype=np.int64)
    n_seq = len(offs) - 1
    lens = np.diff(offs)
    total = int(offs[-1])
    owner = np.repeat(np.arange(n_seq, dtype=np.int64), lens)
    ps = np.broadcast_to(np.asarray(p_sub, dtype=np.float64), (n_seq,))[owner]
    pi = np.broadcast_to(np.asarray(p_ins, dtype=np.float64), (n_seq,))[owner]
    pd = np.broadcast_to(np.asarray(p_del, dtype=np.float64), (n_seq,))[owner]
    u = rng.random(total)
    is_sub = u < ps
    is_ins = (u >= ps) & (u < ps + pi)
    is_del = (u >= ps + pi) & (u < ps + pi + pd)
    shift = rng.integers(1, asz, size=total)
    ins_len = rng.geometric(0.5, size=total)
    del_len = rng.geometric(0.5, size=total)

    pos = np.arange(total, dtype=np.int64)
    ends = np.minimum(pos + del_len, offs[1:][owner])
    delta = np.zeros(total + 1, dtype=np.int64)
    np.add.at(delta, pos[is_del], 1)
    np.add.at(delta, ends[is_del], -1)
    deleted = np.cumsum(delta)[:-1] > 0

    base = np.where(is_sub, (seqs.astype(np.int64) + shift) % asz, seqs).astype(np.uint8)
    n_ins = np.where(is_ins, ins_len, 0)
    keep = ~deleted
    count = n_ins + keep.astype(np.int64)
    slot_end = np.cumsum(count)
    slot_start = slot_end - count
    out = rng.integers(0, asz, size=int(slot_end[-1]) if total else 0, dtype=np.uint8)
    out[slot_start[keep] + n_ins[keep]] = base[keep]
    new_lens = np.bincount(owner, weights=count, minlength=n_seq).astype(np.int64)
    new_offs = np.zeros(n_seq + 1, dtype=np.int64)
    np.cumsum(new_lens, out=new_offs[1:])
    return out, new_offs


def _diverged(rng, seqs, offs, div, asz):
    div = np.asarray(div, dtype=np.float64)
    return mutate(rng, seqs, offs, div / 2, div / 4, div / 4, asz)


# -------------------------------------------------------------- workloads ----

def config0(n_pairs: int = 1000, seed: int = 1000) -> Batch:
    """1,000 pairs, A uniform ACGT^150, B = A with 3% sub, 1% ins, 1% del;
    global affine, match +2, mismatch -3, alpha 5, beta 2."""
    rng = np.random.default_rng(seed)
    sa, oa = random_csr(rng, np.full(n_pairs, 150), 4)
    sb, ob = mutate(rng, sa, oa, 0.03, 0.01, 0.01, 4)
    return Batch("c0: global affine DNA, 150 bp", sa, oa, sb, ob, dna_subst(), 5, 2, MODE_GLOBAL)


def config1(n_pairs: int = 1 << 20, seed: int = 1001) -> Batch:
    """150 bp reads vs 250 bp windows; each window holds its read, mutated with
    5% sub, 1% ins, 1% del (truncated to 250), at a uniform offset; local affine."""
    rng = np.random.default_rng(seed)
    sa, oa = random_csr(rng, np.full(n_pairs, 150), 4)
    rm, ro = mutate(rng, sa, oa, 0.05, 0.01, 0.01, 4)
    rl = np.minimum(np.diff(ro), 250)
    win = rng.integers(0, 4, size=n_pairs * 250, dtype=np.uint8)
    start = rng.integers(0, 250 - rl + 1)
    owner = np.repeat(np.arange(n_pairs, dtype=np.int64), rl)
    within = np.arange(int(rl.sum()), dtype=np.int64) - np.repeat(np.cumsum(rl) - rl, rl)
    win[owner * 250 + start[owner] + within] = rm[ro[:-1][owner] + within]
    ob = np.arange(n_pairs + 1, dtype=np.int64) * 250
    return Batch("c1: local affine DNA, 150 bp reads vs 250 bp windows", sa, oa, win, ob,
                 dna_subst(), 5, 2, MODE_LOCAL)


def config2(n_pairs: int = 100_000, seed: int = 1002, sigma_ln: float = 1.0,
            max_len: int = 20_000) -> Batch:
    """Log-normal lengths (median 1 kb, sigma 1.0, clipped to 50..20,000),
    B from A at divergence U[0, 0.15] (half indels); semi-global affine."""
    rng = np.random.default_rng(seed)
    la = np.clip(np.round(np.exp(rng.normal(math.log(1000.0), sigma_ln, size=n_pairs))),
                 50, max_len).astype(np.int64)
    sa, oa = random_csr(rng, la, 4)
    div = rng.uniform(0.0, 0.15, size=n_pairs)
    sb, ob = _diverged(rng, sa, oa, div, 4)
    return Batch("c2: semi-global affine DNA, log-normal lengths", sa, oa, sb, ob, dna_subst(),
                 5, 2, MODE_SEMIGLOBAL)


def config3(n_pairs: int = 1 << 16, n_long: int = 64, long_len: int = 65536,
            seed: int = 1003) -> Batch:
    """Protein local affine: query U[50,1000] vs target U[50,2000], uniform
    residues, seeded symmetric matrix, alpha 11, beta 1; then n_long pairs of
    long_len residues (first half unrelated, second half B = A at 10%)."""
    rng = np.random.default_rng(seed)
    subst = protein_subst(rng)
    la = rng.integers(50, 1001, size=n_pairs)
    lb = rng.integers(50, 2001, size=n_pairs)
    sa, oa = random_csr(rng, la, 20)
    sb, ob = random_csr(rng, lb, 20)
    if n_long:
        la2, oa2 = random_csr(rng, np.full(n_long, long_len), 20)
        half = n_long // 2
        lb_un, ob_un = random_csr(rng, np.full(half, long_len), 20)
        rel_a = la2[oa2[half]:]
        rel_o = oa2[half:] - oa2[half]
        lb_rel, ob_rel = _diverged(rng, rel_a, rel_o, np.full(n_long - half, 0.10), 20)
        long_b = np.concatenate([lb_un, lb_rel])
        long_ob = np.concatenate([ob_un[:-1], ob_rel + ob_un[-1]])
        sa = np.concatenate([sa, la2])
        oa = np.concatenate([oa[:-1], oa2 + oa[-1]])
        sb = np.concatenate([sb, long_b])
        ob = np.concatenate([ob[:-1], long_ob + ob[-1]])
    return Batch("c3: local affine protein", sa, oa, sb, ob, subst, 11, 1, MODE_LOCAL)


def config4(n_pairs: int = 1_000_000, seed: int = 1004) -> Batch:
    """Lengths U[1000,5000], divergence U[0, 0.10] (half indels); global affine."""
    b = config4_like(n_pairs, seed)
    b.name = "c4: global affine DNA, 1-5 kb"
    return b


def config4_training(n_pairs: int = 200_000, seed: int = 2004) -> Batch:
    """Training pairs for the band network: config 4's law, its own seed."""
    b = config4(n_pairs, seed)
    b.name = "c4 training set"
    return b


def read_set(n_reads: int, length: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """n_reads DNA reads of `length` residues (CSR), drawn at uniform
    positions of a seeded uniform random genome of 2^24 residues, with 0.5%
    substitution errors: a stand-in for the paper's simulated short reads of
    one chromosome aligned all against all (section 4.1), which are not
    available here."""
    rng = np.random.default_rng(seed)
    genome = rng.integers(0, 4, size=1 << 24, dtype=np.uint8)
    starts = rng.integers(0, len(genome) - length + 1, size=n_reads)
    seqs = genome[starts[:, None] + np.arange(length)[None, :]].reshape(-1)
    offs = np.arange(n_reads + 1, dtype=np.int64) * length
    seqs, offs = mutate(rng, seqs, offs, 0.005, 0.0, 0.0, 4)
    return seqs.astype(np.uint8), offs


def random_small(rng: np.random.Generator, n_pairs: int, max_len: int, asz: int = 4,
                 related: float = 0.5) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Mixed small pairs for edge-case tests: lengths U[0, max_len], about
    `related` of them with B derived from A at divergence U[0, 0.3]."""
    la = rng.integers(0, max_len + 1, size=n_pairs)
    sa, oa = random_csr(rng, la, asz)
    div = rng.uniform(0.0, 0.3, size=n_pairs)
    sb_rel, ob_rel = _diverged(rng, sa, oa, div, asz)
    lb = rng.integers(0, max_len + 1, size=n_pairs)
    sb_un, ob_un = random_csr(rng, lb, asz)
    pick = rng.random(n_pairs) < related
    pairs_b = [sb_rel[ob_rel[p]:ob_rel[p + 1]] if pick[p] else sb_un[ob_un[p]:ob_un[p + 1]]
               for p in range(n_pairs)]
    lens_b = np.array([len(x) for x in pairs_b], dtype=np.int64)
    ob = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(lens_b, out=ob[1:])
    sb = np.concatenate(pairs_b) if ob[-1] else np.zeros(0, np.uint8)
    return sa, oa, sb.astype(np.uint8), ob


def config4_like(n_pairs: int, seed: int, min_len: int = 1000, max_len: int = 5000,
                 max_div: float = 0.10) -> Batch:
    """Config 4's law (lengths U[min_len, max_len], divergence U[0, max_div],
    half indels), drawn by the C generator: a million 1-5 kb pairs take
    seconds instead of the numpy path's minutes and tens of GB."""
    rng = np.random.default_rng(seed)
    la = rng.integers(min_len, max_len + 1, size=n_pairs)
    div = rng.uniform(0.0, max_div, size=n_pairs)
    seed_a, seed_b = (int(x) for x in rng.integers(0, 1 << 62, size=2))
    sa, oa = native_csr(seed_a, la, 4)
    sb, ob = native_mutate(seed_b, sa, oa, div / 2, div / 4, div / 4, 4)
    return Batch(f"config-4 law, {min_len}-{max_len} bp", sa, oa, sb, ob, dna_subst(), 5, 2,
                 MODE_GLOBAL)


# ---- random draws of the band network's training (passed to the library as inputs)

# float32 parameter layout of the band network: name -> (offset, shape)
BAND_PARAM_LAYOUT = {"w1": (0, (32, 64)), "b1": (2048, (64,)), "w2": (2112, (64, 64)),
                     "b2": (6208, (64,)), "w3": (6272, (64,)), "b3": (6336, (1,))}
BAND_PARAMS = 6337


def band_params_init(seed: int, b3: float = 0.0) -> np.ndarray:
    """Initial weights: normal with variance 2/fan_in (last layer 1/fan_in),
    zero biases except b3; float32 [6337] in the library's layout."""
    rng = np.random.default_rng(seed)
    p = np.zeros(BAND_PARAMS, dtype=np.float32)
    for name, fan_in, var in (("w1", 32, 2 / 32), ("w2", 64, 2 / 64), ("w3", 64, 1 / 64)):
        off, shape = BAND_PARAM_LAYOUT[name]
        size = int(np.prod(shape))
        p[off:off + size] = rng.normal(0.0, math.sqrt(var), size)
    p[BAND_PARAM_LAYOUT["b3"][0]] = b3
    return p


def band_params_split(flat) -> dict:
    """The flat array as named float32 arrays (views of a copy)."""
    flat = np.asarray(flat, dtype=np.float32).copy()
    return {k: flat[off:off + int(np.prod(shape))].reshape(shape)
            for k, (off, shape) in BAND_PARAM_LAYOUT.items()}


def minibatch_order(seed: int, n: int, n_steps: int, batch: int) -> np.ndarray:
    """Sample indices of n_steps minibatches: consecutive random permutations
    of 0..n-1 (epochs), cut into minibatches of `batch`; int32."""
    rng = np.random.default_rng(seed)
    need = n_steps * batch
    parts, have = [], 0
    while have < need:
        parts.append(rng.permutation(n))
        have += n
    return np.concatenate(parts)[:need].astype(np.int32) if need else np.zeros(0, np.int32)
