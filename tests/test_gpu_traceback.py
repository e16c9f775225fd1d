"""GPU traceback: every returned alignment is an alignment of the pair that
the mode admits (its columns consume exactly the span it reports), its score
recomputed by the oracle's scorer from the definition equals the score the
GPU reports, and that score equals the oracle's optimum.  Several alignments
can be optimal, so the columns themselves are not compared.  The divide and
conquer is forced down to tiny subproblems with the explicit-predecessor
limit lowered from the host, so gap runs crossing split rows, one-row
subproblems and column-less subproblems all occur on small pairs."""
import sys

import numpy as np
import pytest

from paper_2205_07610_amd import synth

pytestmark = pytest.mark.gpu

DNA = synth.dna_subst()


def _say(msg):
    print(f"[traceback] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_07610_amd import binding
    binding.lib()
    return binding


def _check(gpu, oracle_mod, b, label, base=None):
    prev = gpu.set_traceback_base(base) if base is not None else None
    try:
        dev = gpu.to_device(b, "cuda:0")
        sc, ops, span = gpu.align_batch_traceback(*dev, b.subst, b.alpha, b.beta, b.mode)
        sc, ops, span = sc.cpu().numpy(), ops.cpu().numpy(), span.cpu().numpy()
    finally:
        if prev is not None:
            gpu.set_traceback_base(prev)
    _say(f"{label}: {b.n_pairs} pairs, {b.cells():.3g} cells, mode {b.mode}, base {base}")
    want = oracle_mod.align_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, b.subst, b.alpha, b.beta, b.mode)
    bad = np.nonzero(sc.astype(np.int64) != want)[0]
    assert len(bad) == 0, (f"{label}: {len(bad)} score mismatches; pair {bad[0]}: gpu {sc[bad[0]]} oracle "
                           f"{want[bad[0]]} (m={b.lens_a[bad[0]]}, n={b.lens_b[bad[0]]})")
    got = oracle_mod.alignment_score_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, b.subst, b.alpha, b.beta,
                                           b.mode, ops, span)
    bad = np.nonzero(got != want)[0]
    if len(bad):
        p = int(bad[0])
        o = int(b.offs_a[p] - b.offs_a[0] + b.offs_b[p] - b.offs_b[0])
        cols = ops[o:o + max(int(span[p][0]), 0)].tobytes()[:80]
        raise AssertionError(f"{label}: {len(bad)} alignments do not score the optimum; pair {p} "
                             f"(m={b.lens_a[p]}, n={b.lens_b[p]}): alignment scores {got[p]}, optimum "
                             f"{want[p]}, span {span[p].tolist()}, columns {cols!r}")
    # every column count is within m + n and the spans are in range
    assert np.all(span[:, 0] <= b.lens_a + b.lens_b)


def _random_scoring(rng, asz):
    sub = rng.integers(-4, 1, size=(asz, asz))
    sub[np.arange(asz), np.arange(asz)] = rng.integers(1, 4, size=asz)
    sub = sub + np.triu(rng.integers(0, 2, size=(asz, asz)), 1)
    beta = int(rng.integers(0, 4))
    alpha = beta + int(rng.integers(0, 6))
    return sub.astype(np.int8), alpha, beta


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_small_pairs_every_base(gpu, oracle_mod, mode):
    """Random pairs of 0..70 residues, related and unrelated, empty ones
    included, with the explicit-predecessor limit at 1 cell (split down to
    single rows), 40 cells and the default."""
    rng = np.random.default_rng(900 + mode)
    sa, oa, sb, ob = synth.random_small(rng, 300, 70)
    b = synth.Batch("small", sa, oa, sb, ob, DNA, 5, 2, mode)
    for base in (1, 40, None):
        _check(gpu, oracle_mod, b, f"small mode {mode}", base)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_random_scoring_schemes(gpu, oracle_mod, mode):
    """Non-symmetric sigma, linear gaps (alpha == beta), beta == 0, several
    alphabets; split down to single rows and with the default limit."""
    rng = np.random.default_rng(910 + mode)
    for k in range(6):
        asz = int(rng.choice([2, 4, 5, 20]))
        sub, alpha, beta = _random_scoring(rng, asz)
        if k == 0:
            alpha = beta       # linear gaps
        sa, oa, sb, ob = synth.random_small(rng, 120, 90, asz=asz)
        b = synth.Batch("scoring", sa, oa, sb, ob, sub, alpha, beta, mode)
        for base in (1, 300, None):
            _check(gpu, oracle_mod, b, f"scheme {k} asz {asz} a {alpha} b {beta}", base)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_multi_stripe_and_one_row(gpu, oracle_mod, mode):
    """Columns past one 512-column stripe (the stripe hand-off), one-residue
    rows against long columns, long rows against few columns, and pairs
    split many times."""
    rng = np.random.default_rng(920 + mode)
    pairs = []
    for m, n in [(1, 1500), (1, 700), (2, 1300), (3, 2000), (1500, 1), (900, 3), (700, 1100),
                 (1200, 1700), (2100, 600), (513, 513), (512, 1025)]:
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        if rng.random() < 0.6 and m > 3 and n > 3:
            s, _ = synth.mutate(rng, a, np.array([0, m]), 0.08, 0.03, 0.03, 4)
            s = s[:n] if len(s) >= n else np.concatenate([s, rng.integers(0, 4, n - len(s)).astype(np.uint8)])
        else:
            s = rng.integers(0, 4, size=n).astype(np.uint8)
        pairs.append((a, s))
    b = synth.from_pairs("stripes", pairs, DNA, 5, 2, mode)
    for base in (64, None):
        _check(gpu, oracle_mod, b, f"stripes mode {mode}", base)


def test_workload_shapes(gpu, oracle_mod):
    """Sampled pairs of the benchmark workloads: 150 bp global pairs, local
    reads in windows, semi-global pairs of uneven lengths, 1-5 kb global
    pairs and local protein pairs."""
    _check(gpu, oracle_mod, synth.config0(n_pairs=400), "c0")
    c1 = synth.config1(n_pairs=2000)
    _check(gpu, oracle_mod, c1, "c1")
    c2 = synth.config2(n_pairs=3000)
    idx = np.nonzero(np.maximum(c2.lens_a, c2.lens_b) <= 4000)[0][:300]
    _check(gpu, oracle_mod, c2.subset(idx), "c2[300]")
    _check(gpu, oracle_mod, synth.config4_like(64, 930), "c4 law")
    c3 = synth.config3(n_pairs=1 << 16, n_long=0)
    _check(gpu, oracle_mod, c3.subset(np.arange(200)), "c3[200]")


def test_traceback_errors(gpu):
    import torch
    from paper_2205_07610_amd.binding import AlignError
    sa = torch.zeros(10, dtype=torch.uint8, device="cuda")
    ok = torch.tensor([0, 5, 10], dtype=torch.int64, device="cuda")
    bad = torch.tensor([0, 6, 5], dtype=torch.int64, device="cuda")
    with pytest.raises(AlignError) as e:
        gpu.align_batch_traceback(sa, bad, sa, ok, DNA, 5, 2, 0)
    assert e.value.code == -2
    sb = sa.clone()
    sb[7] = 4
    with pytest.raises(AlignError) as e:
        gpu.align_batch_traceback(sa, ok, sb, ok, DNA, 5, 2, 2)
    assert e.value.code == -3
    with pytest.raises(AlignError) as e:
        gpu.align_batch_traceback(sa, ok, sa, ok, DNA, 2, 5, 0)
    assert e.value.code == -4
    sc, ops, span = gpu.align_batch_traceback(sa, ok, sa, ok, DNA, 5, 2, 0)
    assert sc.cpu().tolist() == [10, 10]
    # pair p's columns start at (offs_a[p] - offs_a[0]) + (offs_b[p] - offs_b[0])
    o = ops.cpu().numpy()
    assert o[0:5].tobytes() == b"MMMMM" and o[10:15].tobytes() == b"MMMMM"
    assert span.cpu().tolist() == [[5, 0, 5, 0, 5], [5, 0, 5, 0, 5]]


@pytest.mark.parametrize("length,n_pairs", [(125, 1 << 20), (512, 1 << 17)])
def test_read_pairs_full_size_sampled(gpu, oracle_mod, length, n_pairs):
    """The benchmark's traceback configuration: 2^20 pairs of 125 bp reads
    or 2^17 of 512 bp (3536 reads of a seeded genome, global, linear gaps,
    +2/-1), traced in one call; 3000 sampled pairs have the oracle's optimum
    as their score, and their alignments rescore to it."""
    seqs, offs = synth.read_set(3536, length, 1005 if length == 125 else 1006)
    rng = np.random.default_rng(1007)
    qi, si = rng.integers(0, 3536, size=n_pairs), rng.integers(0, 3536, size=n_pairs)
    b = synth.from_pairs(f"reads {length}", [(seqs[offs[q]:offs[q + 1]], seqs[offs[t]:offs[t + 1]])
                                              for q, t in zip(qi, si)], synth.dna_subst(2, -1), 1, 1, 0)
    dev = gpu.to_device(b, "cuda:0")
    sc, ops, span = gpu.align_batch_traceback(*dev, b.subst, b.alpha, b.beta, b.mode)
    sc, ops, span = sc.cpu().numpy(), ops.cpu().numpy(), span.cpu().numpy()
    _say(f"reads {length}: {n_pairs} pairs traced")
    idx = np.sort(np.random.default_rng(8).choice(n_pairs, size=3000, replace=False))
    sub = b.subset(idx)
    want = oracle_mod.align_batch(sub.seqs_a, sub.offs_a, sub.seqs_b, sub.offs_b, sub.subst, sub.alpha,
                                  sub.beta, sub.mode)
    np.testing.assert_array_equal(sc[idx].astype(np.int64), want)
    # the sampled pairs' columns, gathered from the batch's column buffer
    col0 = (b.offs_a[:-1] - b.offs_a[0]) + (b.offs_b[:-1] - b.offs_b[0])
    sub_ops = np.concatenate([ops[col0[p]:col0[p] + b.lens_a[p] + b.lens_b[p]] for p in idx])
    got = oracle_mod.alignment_score_batch(sub.seqs_a, sub.offs_a, sub.seqs_b, sub.offs_b, sub.subst,
                                           sub.alpha, sub.beta, sub.mode, sub_ops, span[idx])
    np.testing.assert_array_equal(got, want)
