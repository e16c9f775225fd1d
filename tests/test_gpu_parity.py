"""GPU parity: every score from the HIP library equals the CPU oracle's,
bit for bit, on the same seeded inputs.  Runs on an MI355X only."""
import os
import sys

import numpy as np
import pytest

from paper_2205_07610_amd import synth

pytestmark = pytest.mark.gpu

DNA = synth.dna_subst()


def _say(msg):
    print(f"[parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_07610_amd import binding
    binding.lib()
    return binding


def _check(gpu, oracle_mod, batch, label, nthreads=None):
    _say(f"{label}: {batch.n_pairs} pairs, {batch.cells():.3g} cells, mode {batch.mode}")
    got = gpu.align(batch)
    want = oracle_mod.align_batch(batch.seqs_a, batch.offs_a, batch.seqs_b, batch.offs_b,
                                  batch.subst, batch.alpha, batch.beta, batch.mode, nthreads)
    bad = np.nonzero(got.astype(np.int64) != want)[0]
    if len(bad):
        p = int(bad[0])
        raise AssertionError(f"{label}: {len(bad)} mismatches; first pair {p}: gpu {got[p]} oracle "
                             f"{want[p]} (m={batch.lens_a[p]}, n={batch.lens_b[p]})")
    return got


def _oriented(m, n):
    """(rows, columns) as the routing orients a pair of lengths m (A) and n
    (B): the orientation with fewer 256-column stripe passes of (rows + 15)
    steps."""
    sa, sb = (n + 255) // 256, (m + 255) // 256
    return (n, m) if sb * (n + 15) < sa * (m + 15) else (m, n)


def test_config0_all_pairs(gpu, oracle_mod):
    _check(gpu, oracle_mod, synth.config0(), "c0")


def test_config1_subset(gpu, oracle_mod):
    _check(gpu, oracle_mod, synth.config1(n_pairs=8192), "c1[8192]")


def test_config2_subset(gpu, oracle_mod):
    _check(gpu, oracle_mod, synth.config2(n_pairs=2000), "c2[2000]")


def test_config3_subset(gpu, oracle_mod):
    b = synth.config3(n_pairs=400, n_long=2, long_len=3000)
    _check(gpu, oracle_mod, b, "c3[400+2x3000]")


def test_config4_subset(gpu, oracle_mod):
    _check(gpu, oracle_mod, synth.config4(n_pairs=60), "c4[60]")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_small_random_with_empty(gpu, oracle_mod, mode):
    rng = np.random.default_rng(100 + mode)
    sa, oa, sb, ob = synth.random_small(rng, 3000, 40)
    b = synth.Batch("small", sa, oa, sb, ob, DNA, 5, 2, mode)
    _check(gpu, oracle_mod, b, f"small mode {mode}")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_stripe_and_tile_boundaries(gpu, oracle_mod, mode):
    rng = np.random.default_rng(200 + mode)
    pairs = []
    for n in (1, 2, 15, 16, 17, 255, 256, 257, 511, 512, 513, 767, 769, 1000):
        for m in (1, 2, 16, 17, 300):
            a = rng.integers(0, 4, size=m).astype(np.uint8)
            s = rng.integers(0, 4, size=n).astype(np.uint8)
            if rng.random() < 0.5:   # related pair: B contains a mutated copy of A
                k = min(m, n)
                s[:k] = np.where(rng.random(k) < 0.1, rng.integers(0, 4, size=k), a[:k])
            pairs.append((a, s))
            pairs.append((s, a))
    b = synth.from_pairs("bounds", pairs, DNA, 5, 2, mode)
    _check(gpu, oracle_mod, b, f"boundaries mode {mode}")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_asymmetric_sigma_and_gap_variants(gpu, oracle_mod, mode):
    rng = np.random.default_rng(300 + mode)
    sub = rng.integers(-6, 7, size=(5, 5)).astype(np.int8)
    for alpha, beta in [(5, 2), (3, 3), (0, 0), (9, 1), (1, 0)]:
        sa, oa, sb, ob = synth.random_small(rng, 400, 300, asz=5)
        b = synth.Batch("asym", sa, oa, sb, ob, sub, alpha, beta, mode)
        _check(gpu, oracle_mod, b, f"asym sigma a={alpha} b={beta} mode {mode}")


def test_protein_alphabet_and_long_pairs(gpu, oracle_mod):
    rng = np.random.default_rng(400)
    sub = synth.protein_subst(rng)
    pairs = []
    for m, n in [(5000, 4000), (2500, 7000), (64, 9000), (9000, 40)]:
        a = rng.integers(0, 20, size=m).astype(np.uint8)
        s = rng.integers(0, 20, size=n).astype(np.uint8)
        pairs.append((a, s))
    a = rng.integers(0, 20, size=6000).astype(np.uint8)
    pairs.append((a, a.copy()))               # identical: local score = sum of the diagonal
    for mode in (0, 1, 2):
        b = synth.from_pairs("protein long", pairs, sub, 11, 1, mode)
        _check(gpu, oracle_mod, b, f"protein long mode {mode}")


def test_error_codes(gpu):
    import torch
    from paper_2205_07610_amd.binding import AlignError
    sa = torch.zeros(10, dtype=torch.uint8, device="cuda")
    ok = torch.tensor([0, 5, 10], dtype=torch.int64, device="cuda")
    bad = torch.tensor([0, 6, 5], dtype=torch.int64, device="cuda")
    with pytest.raises(AlignError) as e:
        gpu.align_batch(sa, bad, sa, ok, DNA, 5, 2, 0)
    assert e.value.code == -2
    sb = sa.clone()
    sb[7] = 4                                 # code 4 with a 4-letter alphabet
    with pytest.raises(AlignError) as e:
        gpu.align_batch(sa, ok, sb, ok, DNA, 5, 2, 2)
    assert e.value.code == -3
    out = gpu.align_batch(sa, ok, sa, ok, DNA, 5, 2, 2)
    assert out.cpu().tolist() == [10, 10]


def test_packed_lds_local(gpu, oracle_mod):
    """Local pairs of the 32-bit list on packed 16-bit cells with LDS profiles:
    protein pairs of config 3's shapes and DNA pairs wider than one packed
    stripe, two pairs per lane group with unequal lengths and stripe counts,
    then the same batch with the saturation threshold lowered from the host
    so that most pairs are recomputed with 32-bit cells."""
    rng = np.random.default_rng(560)
    c3 = synth.config3(n_pairs=1 << 16, n_long=0)
    idx = np.sort(rng.choice(c3.n_pairs, 1500, replace=False))
    b = c3.subset(idx)
    gpu.enable_timing(True)
    try:
        _check(gpu, oracle_mod, b, "protein local, packed LDS")
        tm = gpu.last_timing()
    finally:
        gpu.enable_timing(False)
    assert tm["pairs_full32"] == b.n_pairs and tm["pairs_rerun32"] == 0
    prev = gpu.set_i16_limit(40)
    try:
        _check(gpu, oracle_mod, b.subset(np.arange(400)), "protein local, forced re-run")
    finally:
        gpu.set_i16_limit(prev)
    pairs = []
    for k in range(160):
        m, n = (int(x) for x in rng.integers(1, 1500, size=2))
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        if k % 2:
            s_, _ = synth.mutate(rng, a, np.array([0, m]), 0.05, 0.02, 0.02, 4)
            s_ = s_[:n] if len(s_) >= n else np.concatenate([s_, rng.integers(0, 4, n - len(s_)).astype(np.uint8)])
        else:
            s_ = rng.integers(0, 4, size=n).astype(np.uint8)
        pairs.append((a, s_))
    _check(gpu, oracle_mod, synth.from_pairs("dna local", pairs, DNA, 5, 2, 2), "DNA local, mixed routes")


def test_local_scores_beyond_int16(gpu, oracle_mod):
    """Local DNA pairs of 300-1200 residues with match 100 (mismatch -20,
    alpha 20, beta 5): identical and nearly identical pairs score up to
    120,000, far past int16, so the packed LDS-profile kernel saturates on
    its own (no lowered threshold) and the 32-bit re-run gives the exact
    scores; unrelated pairs stay on 16-bit cells."""
    rng = np.random.default_rng(570)
    sub = synth.dna_subst(100, -20)
    pairs = []
    for k in range(120):
        m = int(rng.integers(300, 1201))
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        if k % 3 == 0:
            s_ = a.copy()
        elif k % 3 == 1:
            s_, _ = synth.mutate(rng, a, np.array([0, m]), 0.02, 0.005, 0.005, 4)
            s_ = s_.astype(np.uint8)
        else:
            s_ = rng.integers(0, 4, size=int(rng.integers(300, 1201))).astype(np.uint8)
        pairs.append((a, s_))
    b = synth.from_pairs("local beyond int16", pairs, sub, 20, 5, 2)
    gpu.enable_timing(True)
    try:
        got = _check(gpu, oracle_mod, b, "local beyond int16")
        tm = gpu.last_timing()
    finally:
        gpu.enable_timing(False)
    assert got.max() > 32767
    assert tm["pairs_rerun32"] >= 40


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_all_mismatch_and_very_unequal_lengths(gpu, oracle_mod, mode):
    """Pairs with no matching letter at all (A all 0, B all 1, 1..3000
    residues), and very unequal lengths in both orientations (1-10 residues
    against 3000-20000, and the reverse): global scores run deep negative
    (down to about -40,000), local and semi-global ones sit at their floors;
    every route (packed, 32-bit stripes, wavefront) meets them."""
    rng = np.random.default_rng(580 + mode)
    pairs = []
    for _ in range(60):
        m, n = (int(x) for x in rng.integers(1, 3001, size=2))
        pairs.append((np.zeros(m, np.uint8), np.ones(n, np.uint8)))
    for _ in range(40):
        short = rng.integers(0, 4, size=int(rng.integers(1, 11))).astype(np.uint8)
        long_ = rng.integers(0, 4, size=int(rng.integers(3000, 20001))).astype(np.uint8)
        pairs.append((short, long_) if rng.random() < 0.5 else (long_, short))
    b = synth.from_pairs("adversarial", pairs, DNA, 5, 2, mode)
    got = _check(gpu, oracle_mod, b, f"all-mismatch and unequal, mode {mode}")
    if mode == 0:
        assert got.min() < -30000


def test_range_refusal(gpu):
    """AS_ERR_RANGE: a pair whose cells could leave the 32-bit budget is
    refused before any DP runs (|sigma|max + alpha + 2 beta) * (m + n + 2)
    >= 2^28; with alpha = beta = 60 on DNA that is m + n >= 1.47 M.  The
    same batch one residue shorter on each side of that line is accepted by
    the check (not aligned here: the other pair is empty)."""
    import torch
    from paper_2205_07610_amd.binding import AlignError
    budget = 1 << 28
    per = 3 + 60 + 2 * 60
    m = (budget + per - 1) // per - 2          # smallest m + n (split evenly) that is refused
    half = (m + 1) // 2
    seq = torch.zeros(half, dtype=torch.uint8, device="cuda")
    oa = torch.tensor([0, half], dtype=torch.int64, device="cuda")
    ob = torch.tensor([0, m - half], dtype=torch.int64, device="cuda")
    with pytest.raises(AlignError) as e:
        gpu.align_batch(seq, oa, seq, ob, DNA, 60, 60, 0)
    assert e.value.code == -5
    # an empty pair of the same total length is scored by its closed form only
    # when the range check passes: one residue less passes it
    ok_a = torch.tensor([0, 0], dtype=torch.int64, device="cuda")
    ok_b = torch.tensor([0, m - 1], dtype=torch.int64, device="cuda")
    big = torch.zeros(m - 1, dtype=torch.uint8, device="cuda")
    out = gpu.align_batch(seq, ok_a, big, ok_b, DNA, 60, 60, 0)
    assert out.cpu().tolist() == [-60 - 60 * (m - 2)]


def test_deterministic(gpu):
    b = synth.config1(n_pairs=4096, seed=77)
    r1 = gpu.align(b)
    r2 = gpu.align(b)
    assert np.array_equal(r1, r2)


def test_config1_full_size_sampled(gpu, oracle_mod):
    """All 2^20 pairs in the benchmark's configuration; 3000 sampled pairs
    are checked against the oracle, every score against its bounds."""
    b = synth.config1()
    _say(f"c1 full: {b.n_pairs} pairs")
    got = gpu.align(b)
    assert got.min() >= 0 and got.max() <= 2 * 150
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(b.n_pairs, size=3000, replace=False))
    sub = b.subset(idx)
    want = oracle_mod.align_batch(sub.seqs_a, sub.offs_a, sub.seqs_b, sub.offs_b, sub.subst,
                                  sub.alpha, sub.beta, sub.mode)
    assert np.array_equal(got[idx].astype(np.int64), want)


def _full_size_sampled(gpu, oracle_mod, b, label, n_sample, seed):
    _say(f"{label}: {b.n_pairs} pairs, {b.cells():.3g} cells, mode {b.mode}")
    got = gpu.align(b)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(b.n_pairs, size=n_sample, replace=False))
    sub = b.subset(idx)
    want = oracle_mod.align_batch(sub.seqs_a, sub.offs_a, sub.seqs_b, sub.offs_b, sub.subst,
                                  sub.alpha, sub.beta, sub.mode)
    bad = np.nonzero(got[idx].astype(np.int64) != want)[0]
    assert len(bad) == 0, f"{label}: {len(bad)} of {n_sample} sampled pairs differ (first {idx[bad[0]]})"
    return got


def test_config2_full_size_sampled(gpu, oracle_mod):
    """All 10^5 semi-global pairs of log-normal length (50..20,000) in the
    benchmark's configuration; 2000 sampled pairs checked against the
    oracle, and every score is at least the empty alignment's 0 and at most
    sigma_max times the shorter length."""
    b = synth.config2()
    got = _full_size_sampled(gpu, oracle_mod, b, "c2 full", 2000, 6)
    assert got.min() >= 0
    assert np.all(got.astype(np.int64) <= 2 * np.minimum(b.lens_a, b.lens_b))


def test_config3_short_full_size_sampled(gpu, oracle_mod):
    """All 2^16 short local protein pairs (packed LDS-profile variant and
    the 32-bit re-run); 3000 sampled pairs checked against the oracle."""
    b = synth.config3(n_long=0)
    got = _full_size_sampled(gpu, oracle_mod, b, "c3 short full", 3000, 7)
    assert got.min() >= 0


def test_config4_full_dp_sampled(gpu, oracle_mod):
    """The full DP of all 10^6 pairs of 1-5 kb (packed wavefront, the
    learned path's reference); 1500 sampled pairs checked against the
    oracle."""
    b = synth.config4()
    _full_size_sampled(gpu, oracle_mod, b, "c4 full DP", 1500, 8)


def test_packed16_rerun_forced(gpu, oracle_mod):
    """Lowering the 16-bit saturation threshold from the host sends pairs
    through the 32-bit re-run; scores stay exact and the re-run is used."""
    b = synth.config1(n_pairs=5000, seed=91)
    prev = gpu.set_i16_limit(200)
    try:
        gpu.enable_timing(True)
        got = _check(gpu, oracle_mod, b, "c1 rerun forced")
        tm = gpu.last_timing()
    finally:
        gpu.set_i16_limit(prev)
        gpu.enable_timing(False)
    assert tm["pairs_full16"] == b.n_pairs
    assert tm["pairs_rerun32"] == int(np.count_nonzero(got >= 200)) > 0


def test_packed16_routing(gpu, oracle_mod):
    """Short DNA pairs take the packed path in every mode; unequal row counts
    inside one packed group are handled."""
    rng = np.random.default_rng(92)
    for mode in (0, 1, 2):
        sa, oa, sb, ob = synth.random_small(rng, 4000, 250)
        b = synth.Batch("pk", sa, oa, sb, ob, DNA, 5, 2, mode)
        gpu.enable_timing(True)
        try:
            _check(gpu, oracle_mod, b, f"packed routing mode {mode}")
            tm = gpu.last_timing()
        finally:
            gpu.enable_timing(False)
        assert tm["pairs_full16"] > 0.9 * b.n_pairs


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_wavefront_long_pairs(gpu, oracle_mod, mode):
    """Pairs long enough for the multi-wave wavefront: many stripes, ragged
    last stripe, both orientations, related and unrelated."""
    rng = np.random.default_rng(500 + mode)
    pairs = []
    for m, n in [(2048, 1025), (3000, 5000), (7000, 2100), (4097, 4097), (2500, 9999)]:
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        if rng.random() < 0.5:
            s, _ = synth.mutate(rng, a, np.array([0, m]), 0.05, 0.02, 0.02, 4)
            s = s[:n] if len(s) >= n else np.concatenate([s, rng.integers(0, 4, n - len(s)).astype(np.uint8)])
        else:
            s = rng.integers(0, 4, size=n).astype(np.uint8)
        pairs.append((a, s))
    b = synth.from_pairs("wavefront", pairs, DNA, 5, 2, mode)
    gpu.enable_timing(True)
    try:
        _check(gpu, oracle_mod, b, f"wavefront mode {mode}")
        tm = gpu.last_timing()
    finally:
        gpu.enable_timing(False)
    # (2048, 1025) is oriented with 1025 rows: the packed wavefront takes it
    # in global mode (from 1024 rows), the 32-bit wavefront does not (2048);
    # in global mode every pair fits the packed wavefront's range proof
    if mode == 0:
        assert tm["pairs_long16"] == len(pairs) and tm["pairs_long"] == 0
    else:
        assert tm["pairs_long"] == len(pairs) - 1 and tm["pairs_long16"] == 0


def test_packed_wavefront_duos(gpu, oracle_mod):
    """Global long pairs on the packed wavefront: an odd number of pairs (the
    last duo has one half), duos whose halves differ in stripe and row
    counts, both orientations, related and unrelated pairs, and one pair
    beyond the int16 range proof that stays on the 32-bit wavefront."""
    rng = np.random.default_rng(530)
    pairs = []
    for k in range(36):
        m = int(rng.integers(2048, 4600))
        n = int(rng.integers(1025, 5200))
        if k % 3 == 0:
            m, n = n + 1100, m  # rows from B
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        if k % 2:
            s, _ = synth.mutate(rng, a, np.array([0, m]), 0.06, 0.02, 0.02, 4)
            s = s[:n] if len(s) >= n else np.concatenate([s, rng.integers(0, 4, n - len(s)).astype(np.uint8)])
        else:
            s = rng.integers(0, 4, size=n).astype(np.uint8)
        pairs.append((a, s))
    big = rng.integers(0, 4, size=8200).astype(np.uint8)
    sbig, _ = synth.mutate(rng, big, np.array([0, 8200]), 0.03, 0.01, 0.01, 4)
    pairs.append((big, sbig))
    b = synth.from_pairs("packed wavefront", pairs, DNA, 5, 2, 0)
    gpu.enable_timing(True)
    try:
        _check(gpu, oracle_mod, b, "packed wavefront duos")
        tm = gpu.last_timing()
    finally:
        gpu.enable_timing(False)
    _say(f"packed wavefront: {tm['pairs_long16']} pairs in {tm['long16_ms']:.2f} ms, "
         f"32-bit wavefront {tm['pairs_long']}")
    # packed wavefront pairs have at least 1024 rows and more than 1024 columns
    def wavefront(m, n):
        rows, cols = _oriented(m, n)
        return rows >= 1024 and cols > 1024
    expect = sum(wavefront(len(a), len(s)) for a, s in pairs[:-1])
    assert expect >= 20
    assert tm["pairs_long16"] == expect and tm["pairs_long"] == 1


def test_packed_wavefront_stripe_widths(gpu, oracle_mod):
    """Packed wavefront duos whose stripes narrow to 64 K columns, K = 11..16,
    over 3 to 6 stripes: column counts just past a multiple of 1024 (the
    narrowest K for their stripe count), in between, and exact multiples;
    halves of one duo with different stripe and row counts."""
    rng = np.random.default_rng(540)
    lens = [2049, 2112, 2113, 2400, 2600, 2800, 3072, 3073, 3500, 4096, 4097, 4500, 5120, 5121]
    pairs = []
    for k, L in enumerate(lens):
        for rel in (0, 1):
            m = L + int(rng.integers(0, 24))
            a = rng.integers(0, 4, size=m).astype(np.uint8)
            if rel:
                s, _ = synth.mutate(rng, a, np.array([0, m]), 0.05, 0.02, 0.02, 4)
                s = s[:L] if len(s) >= L else np.concatenate([s, rng.integers(0, 4, L - len(s)).astype(np.uint8)])
            else:
                s = rng.integers(0, 4, size=L).astype(np.uint8)
            pairs.append((a, s) if k % 2 else (s, a))
    b = synth.from_pairs("packed wavefront widths", pairs, DNA, 5, 2, 0)
    gpu.enable_timing(True)
    try:
        _check(gpu, oracle_mod, b, "packed wavefront stripe widths")
        tm = gpu.last_timing()
    finally:
        gpu.enable_timing(False)
    assert tm["pairs_long16"] == len(pairs) and tm["pairs_long"] == 0
    # registers per lane of each pair alone: the smallest K whose 1024-column
    # stripe count of 64 K columns covers its columns
    def k_of(m, n):
        cols = _oriented(m, n)[1]
        S = -(-cols // 1024)
        return max(10, -(-cols // (64 * S)))
    ks = {k_of(len(a), len(s)) for a, s in pairs}
    assert ks >= {11, 12, 13, 14, 15, 16}


def test_config3_long_pairs_full_size_sampled(gpu, oracle_mod):
    """The 64 pairs of 65,536 residues in the benchmark configuration; four of
    them (two unrelated, two related) are checked against the oracle."""
    b = synth.config3(n_pairs=0, n_long=64, long_len=65536)
    _say(f"c3 long: {b.n_pairs} pairs, {b.cells():.3g} cells")
    gpu.enable_timing(True)
    try:
        got = gpu.align(b)
        tm = gpu.last_timing()
    finally:
        gpu.enable_timing(False)
    _say(f"c3 long: wavefront {tm['long_ms']:.1f} ms, {b.cells() / tm['long_ms'] / 1e9:.1f} TCUPS")
    idx = np.array([0, 1, 32, 33])
    sub = b.subset(idx)
    want = oracle_mod.align_batch(sub.seqs_a, sub.offs_a, sub.seqs_b, sub.offs_b, sub.subst,
                                  sub.alpha, sub.beta, sub.mode, nthreads=4)
    assert np.array_equal(got[idx].astype(np.int64), want)
    assert got.min() >= 0
