"""All-against-all batches: every (query, subject) score equals the oracle's
for the same pair, on the implicit-pair packed kernel (one set fitting one
packed stripe, either set) and on the chunked path through the ordinary
routing (both sets longer, protein alphabet, failed range proof), in every
mode, with empty sequences and the forced 32-bit re-run."""
import sys

import numpy as np
import pytest

from paper_2205_07610_amd import synth

pytestmark = pytest.mark.gpu

DNA = synth.dna_subst()


def _say(msg):
    print(f"[all-vs-all] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_07610_amd import binding
    binding.lib()
    return binding


def _set(rng, n, lo, hi, asz=4, base=None, related=0.0):
    """n sequences of lengths U[lo, hi]; a share of them mutated copies of
    `base` sequences (so some pairs are similar)."""
    seqs = []
    for i in range(n):
        if base is not None and rng.random() < related:
            a = base[int(rng.integers(0, len(base)))]
            if len(a):
                b, _ = synth.mutate(rng, a, np.array([0, len(a)]), 0.04, 0.01, 0.01, asz)
                seqs.append(b.astype(np.uint8)[:hi])
                continue
        seqs.append(rng.integers(0, asz, size=int(rng.integers(lo, hi + 1))).astype(np.uint8))
    return seqs


def _csr(seqs):
    offs = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum([len(x) for x in seqs], out=offs[1:])
    data = np.concatenate(seqs) if offs[-1] else np.zeros(0, np.uint8)
    return data.astype(np.uint8), offs


def _check(gpu, oracle_mod, Q, S, subst, alpha, beta, mode, label):
    import torch
    sq, oq = _csr(Q)
    ss, os_ = _csr(S)
    t = lambda x: torch.from_numpy(x).cuda()
    got = gpu.align_all_vs_all(t(sq), t(oq), t(ss), t(os_), subst, alpha, beta, mode).cpu().numpy()
    pairs = [(q, s) for q in Q for s in S]
    b = synth.from_pairs("avsa", pairs, subst, alpha, beta, mode)
    want = oracle_mod.align_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, b.subst, b.alpha, b.beta,
                                  b.mode).reshape(len(Q), len(S))
    bad = np.argwhere(got.astype(np.int64) != want)
    _say(f"{label}: {len(Q)} x {len(S)} pairs, mode {mode}, {len(bad)} mismatches")
    if len(bad):
        q, s = bad[0]
        raise AssertionError(f"{label}: {len(bad)} mismatches; query {q} (len {len(Q[q])}) vs subject {s} "
                             f"(len {len(S[s])}): gpu {got[q, s]} oracle {want[q, s]}")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_short_subjects_packed(gpu, oracle_mod, mode):
    """Subjects fit one packed stripe: queries of any length stream through
    each subject's profile; empty sequences on both sides."""
    rng = np.random.default_rng(1100 + mode)
    Q = _set(rng, 41, 0, 420)
    S = _set(rng, 27, 0, 256, base=Q, related=0.4)
    Q[3] = np.zeros(0, np.uint8)
    S[5] = np.zeros(0, np.uint8)
    _check(gpu, oracle_mod, Q, S, DNA, 5, 2, mode, "short subjects")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_short_queries_transposed(gpu, oracle_mod, mode):
    """Only the queries fit one stripe: the queries become the profile side,
    with an asymmetric sigma so the orientation of sigma matters."""
    rng = np.random.default_rng(1110 + mode)
    sub = np.array([[3, -2, -1, -4], [-3, 2, -4, -1], [0, -4, 1, -2], [-4, -1, -3, 2]], dtype=np.int8)
    Q = _set(rng, 30, 1, 200)
    S = _set(rng, 19, 260, 700, base=Q, related=0.3)
    _check(gpu, oracle_mod, Q, S, sub, 6, 1, mode, "short queries")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_long_sets_chunked_path(gpu, oracle_mod, mode):
    """Both sets longer than a stripe: descriptors through the ordinary
    routing (32-bit stripes, wavefronts for the longest)."""
    rng = np.random.default_rng(1120 + mode)
    Q = _set(rng, 9, 257, 2600)
    S = _set(rng, 7, 257, 2400, base=Q, related=0.5)
    _check(gpu, oracle_mod, Q, S, DNA, 5, 2, mode, "long sets")


def test_protein_and_linear_gaps(gpu, oracle_mod):
    rng = np.random.default_rng(1130)
    sub = synth.protein_subst(rng)
    Q = _set(rng, 17, 0, 300, asz=20)
    S = _set(rng, 13, 1, 200, asz=20, base=Q, related=0.4)
    _check(gpu, oracle_mod, Q, S, sub, 11, 1, 2, "protein local")
    Q = _set(rng, 23, 0, 150)
    S = _set(rng, 21, 0, 150, base=Q, related=0.5)
    _check(gpu, oracle_mod, Q, S, DNA, 3, 3, 0, "linear gaps")


def test_forced_rerun_local(gpu, oracle_mod):
    """The saturation threshold lowered from the host sends most local pairs
    of the packed all-against-all kernel to the 32-bit re-run."""
    rng = np.random.default_rng(1140)
    Q = _set(rng, 33, 1, 300)
    S = _set(rng, 18, 1, 250, base=Q, related=0.6)
    prev = gpu.set_i16_limit(60)
    try:
        _check(gpu, oracle_mod, Q, S, DNA, 5, 2, 2, "forced re-run")
    finally:
        gpu.set_i16_limit(prev)


def test_all_vs_all_errors(gpu):
    import torch
    from paper_2205_07610_amd.binding import AlignError
    seq = torch.zeros(10, dtype=torch.uint8, device="cuda")
    ok = torch.tensor([0, 5, 10], dtype=torch.int64, device="cuda")
    bad = torch.tensor([0, 6, 5], dtype=torch.int64, device="cuda")
    with pytest.raises(AlignError) as e:
        gpu.align_all_vs_all(seq, bad, seq, ok, DNA, 5, 2, 0)
    assert e.value.code == -2
    s2 = seq.clone()
    s2[7] = 9
    with pytest.raises(AlignError) as e:
        gpu.align_all_vs_all(seq, ok, s2, ok, DNA, 5, 2, 2)
    assert e.value.code == -3
    out = gpu.align_all_vs_all(seq, ok, seq, ok, DNA, 5, 2, 2)
    assert out.cpu().tolist() == [[10, 10], [10, 10]]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_half_cells(gpu, oracle_mod, mode):
    """FP16 cells in the all-against-all packed kernel (forced where the
    scoring admits them): DNA scoring takes E4M3 profile bytes in global and
    semi-global mode and E5M2 in local mode (rows of at most 200 residues
    keep global and semi-global cells under the FP16 row bound); then local
    with the re-run threshold lowered from the host."""
    rng = np.random.default_rng(1150 + mode)
    Q = _set(rng, 37, 0, 200)
    S = _set(rng, 29, 0, 256, base=Q, related=0.5)
    prev = gpu.set_half_cells(1)
    prev_t = gpu.enable_timing(True)
    try:
        _check(gpu, oracle_mod, Q, S, DNA, 5, 2, mode, "half cells")
        t = gpu.last_timing()
        assert t["full16_cell_type"] == (2 if mode == 2 else 1), t["full16_cell_type"]
        if mode == 2:
            prev_l = gpu.set_i16_limit(60)
            try:
                _check(gpu, oracle_mod, Q, S, DNA, 5, 2, mode, "half cells, forced re-run")
                assert gpu.last_timing()["pairs_full16"] < len(Q) * len(S)
            finally:
                gpu.set_i16_limit(prev_l)
    finally:
        gpu.enable_timing(prev_t)
        gpu.set_half_cells(prev)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_short_columns_128(gpu, oracle_mod, mode):
    """Column sequences of at most 128 residues take 128-column stripes:
    subjects of 0..128 against queries of any length (int16 and FP16
    cells), and the transposed case with queries of 1..128 against long
    subjects."""
    rng = np.random.default_rng(1160 + mode)
    Q = _set(rng, 35, 0, 300)
    S = _set(rng, 31, 0, 128, base=Q, related=0.4)
    S[4] = np.zeros(0, np.uint8)
    _check(gpu, oracle_mod, Q, S, DNA, 5, 2, mode, "columns <= 128")
    prev = gpu.set_half_cells(1)
    try:
        _check(gpu, oracle_mod, Q[:20], S, synth.dna_subst(1, -1), 3, 1, mode, "columns <= 128, FP16")
    finally:
        gpu.set_half_cells(prev)
    Q2 = _set(rng, 19, 1, 128)
    S2 = _set(rng, 13, 300, 900, base=Q2, related=0.3)
    _check(gpu, oracle_mod, Q2, S2, DNA, 5, 2, mode, "queries <= 128 transposed")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_columns_512(gpu, oracle_mod, mode):
    """The shorter set's sequences of 257..512 residues take 512-column
    stripes (K = 32), either set as columns; local pairs forced to the
    32-bit re-run keep their 512 columns in one stripe."""
    rng = np.random.default_rng(1170 + mode)
    Q = _set(rng, 23, 300, 700)
    S = _set(rng, 17, 257, 512, base=Q, related=0.5)
    _check(gpu, oracle_mod, Q, S, DNA, 5, 2, mode, "columns <= 512")
    Q2 = _set(rng, 15, 100, 512)
    S2 = _set(rng, 21, 513, 800, base=Q2, related=0.3)
    _check(gpu, oracle_mod, Q2, S2, DNA, 5, 2, mode, "queries as columns")
    if mode == 2:
        prev = gpu.set_i16_limit(60)
        try:
            _check(gpu, oracle_mod, Q, S, DNA, 5, 2, mode, "columns <= 512, forced re-run")
        finally:
            gpu.set_i16_limit(prev)


@pytest.mark.parametrize("length", [125, 512])
def test_read_sets_full_size_sampled(gpu, oracle_mod, length):
    """The benchmark's configuration: 3536 reads of 125 or 512 bp all
    against all (12.5 M pairs, global, linear gaps, +2/-1) in one call; 3000
    sampled (query, subject) scores equal the oracle's, and the matrix is
    symmetric (the set against itself, a symmetric scoring)."""
    import torch
    seqs, offs = synth.read_set(3536, length, 1005 if length == 125 else 1006)
    sq, oq = torch.from_numpy(seqs).cuda(), torch.from_numpy(offs).cuda()
    sub = synth.dna_subst(2, -1)
    got = gpu.align_all_vs_all(sq, oq, sq, oq, sub, 1, 1, 0).cpu().numpy()
    _say(f"reads {length}: 3536 x 3536 scored")
    assert np.array_equal(got, got.T)
    rng = np.random.default_rng(9)
    qi, si = rng.integers(0, 3536, 3000), rng.integers(0, 3536, 3000)
    b = synth.from_pairs("sample", [(seqs[offs[q]:offs[q + 1]], seqs[offs[s]:offs[s + 1]]) for q, s in zip(qi, si)],
                         sub, 1, 1, 0)
    want = oracle_mod.align_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, b.subst, b.alpha, b.beta, b.mode)
    np.testing.assert_array_equal(got[qi, si].astype(np.int64), want)


@pytest.mark.parametrize("m", [1, 2, 15, 16, 17, 100, 300])
def test_equal_length_rows_streamed(gpu, oracle_mod, m):
    """Global calls whose row sequences all have one length stream them
    through the packed pipeline without draining it between pairs: rows of
    m residues (a ragged count, so the last block and group run short)
    against columns of 1-500 residues (every stripe width), in both
    orientations, with int16 and FP16 cells; every score equals the
    oracle's."""
    rng = np.random.default_rng(1500 + m)
    n_rows = 37
    rows = [rng.integers(0, 4, size=m).astype(np.uint8) for _ in range(n_rows)]
    for i in range(0, n_rows, 4):  # some rows related to the first column
        rows[i] = rows[0].copy()
    for col_max in (120, 250, 500):
        cols = _set(rng, 13, 1, col_max, base=rows, related=0.3)
        for hmode in (0, 1):
            prev = gpu.set_half_cells(hmode)
            try:
                # rows as queries (columns are the subjects), then as subjects
                _check(gpu, oracle_mod, rows, cols, DNA, 5, 2, 0, f"rows {m} cols {col_max} half {hmode}")
                _check(gpu, oracle_mod, cols, rows, DNA, 5, 2, 0, f"rows {m} (transposed) cols {col_max}")
            finally:
                gpu.set_half_cells(prev)
    # linear gaps with the paper's read scoring
    _check(gpu, oracle_mod, rows, _set(rng, 9, 1, 128), synth.dna_subst(2, -1), 1, 1, 0, f"rows {m} linear")
