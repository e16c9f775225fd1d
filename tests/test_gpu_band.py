"""GPU parity of the banded path: raw banded scores against the oracle's DP
restricted to the same diagonals (the limits the kernel reports), and the
certified path's final scores against the oracle's full DP."""
import sys

import numpy as np
import pytest

from paper_2205_07610_amd import synth

pytestmark = pytest.mark.gpu

DNA = synth.dna_subst()


def _say(msg):
    print(f"[band] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_07610_amd import binding
    binding.lib()
    return binding


def _dev(b):
    from paper_2205_07610_amd import binding
    return binding.to_device(b)


def _w(torch, w):
    return torch.as_tensor(np.asarray(w, dtype=np.int32)).to("cuda")


def _pairs_mixed(rng, n_pairs, max_len, related=0.7):
    sa, oa, sb, ob = synth.random_small(rng, n_pairs, max_len, related=related)
    return sa, oa, sb, ob


@pytest.mark.parametrize("mode", [0, 1])
def test_raw_band_scores_match_oracle(gpu, oracle_mod, mode):
    import torch
    rng = np.random.default_rng(700 + mode)
    sa, oa, sb, ob = _pairs_mixed(rng, 1500, 700)
    b = synth.Batch("band raw", sa, oa, sb, ob, DNA, 5, 2, mode)
    m, n = b.lens_a, b.lens_b
    # half-widths of every class, kept within the widest band (1024 diagonals)
    w = rng.integers(0, 60, size=b.n_pairs)
    w[::7] = 0
    w[::11] = rng.integers(100, 300, size=len(w[::11]))
    w = np.minimum(w, np.maximum(0, (1024 - 1 - np.abs(n - m)) // 2))
    keep = np.abs(n - m) + 2 * w + 1 <= 1024
    b = b.subset(np.nonzero(keep)[0])
    w = w[keep]
    _say(f"raw mode {mode}: {b.n_pairs} pairs")
    got, lo, hi = gpu.band_scores(*_dev(b), b.subst, b.alpha, b.beta, b.mode, _w(torch, w))
    got, lo, hi = got.cpu().numpy(), lo.cpu().numpy(), hi.cpu().numpy()
    ne = (b.lens_a > 0) & (b.lens_b > 0)
    # every computed band contains the requested one and is at most 1024 wide
    L = np.minimum(0, b.lens_b - b.lens_a) - w
    U = np.maximum(0, b.lens_b - b.lens_a) + w
    assert np.all(lo[ne] <= L[ne]) and np.all(hi[ne] >= U[ne]) and np.all(hi[ne] - lo[ne] < 1024)
    idx = np.nonzero(ne)[0]
    sub = b.subset(idx)
    want = oracle_mod.diag_band_batch(sub.seqs_a, sub.offs_a, sub.seqs_b, sub.offs_b, sub.subst,
                                      sub.alpha, sub.beta, sub.mode, lo[idx], hi[idx])
    bad = np.nonzero(got[idx].astype(np.int64) != want)[0]
    assert len(bad) == 0, (f"{len(bad)} mismatches, first pair {idx[bad[0]]}: gpu {got[idx[bad[0]]]} "
                           f"oracle {want[bad[0]]} m={sub.lens_a[bad[0]]} n={sub.lens_b[bad[0]]} "
                           f"lo={lo[idx[bad[0]]]} hi={hi[idx[bad[0]]]}")


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("w0,rounds", [(0, 6), (8, 6), (40, 1), (3, 2)])
def test_certified_band_equals_full(gpu, oracle_mod, mode, w0, rounds):
    import torch
    rng = np.random.default_rng(800 + 10 * mode + w0 + rounds)
    b = synth.config4(n_pairs=150, seed=int(rng.integers(1 << 30)))
    b.mode = mode
    extra = synth.random_small(rng, 300, 400, related=0.8)
    b2 = synth.Batch("mixed", *extra, DNA, 5, 2, mode)
    idx_all = [b, b2]
    pairs = []
    for bb in idx_all:
        for p in range(bb.n_pairs):
            pairs.append(bb.pair(p))
    batch = synth.from_pairs("band cert", pairs, DNA, 5, 2, mode)
    _say(f"certified mode {mode} w0={w0} rounds={rounds}: {batch.n_pairs} pairs")
    got, stats = gpu.align_batch_band(*_dev(batch), batch.subst, batch.alpha, batch.beta,
                                      batch.mode, _w(torch, np.full(batch.n_pairs, w0)),
                                      max_rounds=rounds)
    want = oracle_mod.align_batch(batch.seqs_a, batch.offs_a, batch.seqs_b, batch.offs_b,
                                  batch.subst, batch.alpha, batch.beta, batch.mode)
    got = got.cpu().numpy().astype(np.int64)
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[0]}: {got[bad[0]]} vs {want[bad[0]]}"
    nonempty = int(np.count_nonzero((batch.lens_a > 0) & (batch.lens_b > 0)))
    assert sum(stats["accepted"]) + stats["fallback"] == nonempty
    _say(f"  stats {stats}")


def test_band_api_errors(gpu):
    import torch
    from paper_2205_07610_amd.binding import AlignError
    b = synth.config0(n_pairs=10)
    with pytest.raises(AlignError) as e:                 # local mode has no band path
        gpu.align_batch_band(*_dev(b), b.subst, 5, 2, 2, _w(torch, np.zeros(10)))
    assert e.value.code == -7
    with pytest.raises(AlignError) as e:                 # band wider than 1536 diagonals
        gpu.band_scores(*_dev(b), b.subst, 5, 2, 0, _w(torch, np.full(10, 800)))
    assert e.value.code == -7
    with pytest.raises(AlignError) as e:                 # exact band wider than 1024 diagonals
        gpu.band_certify(*_dev(b), b.subst, 5, 2, 0, _w(torch, np.full(10, 600)))
    assert e.value.code == -7
    prot = synth.protein_subst(np.random.default_rng(1))
    pb = synth.config3(n_pairs=4, n_long=0)
    with pytest.raises(AlignError) as e:                 # 20-letter alphabet
        gpu.align_batch_band(*_dev(pb), prot, 11, 1, 0, _w(torch, np.zeros(4)))
    assert e.value.code == -4


def test_packed_band_matches_32bit_and_oracle(gpu, oracle_mod):
    """Global certified banding with the packed 16-bit kernel on (default)
    and off: both equal the oracle's full DP for every pair.  Pairs of ~4900
    and ~6000 residues need the packed kernel's lowered bias (their upper
    bound passes 32768), initial half-widths
    range from 0 to wide, so pairs are accepted, doubled and sent to the
    full DP; one case spreads the initial widths over every class.  The
    packed classes of 96, 192, 384 and 768 diagonals (K = 6 or 12 registers
    per lane) run their selector rotation in three phases."""
    import torch
    rng = np.random.default_rng(760)
    b = synth.config4_like(900, 761, min_len=150, max_len=2500, max_div=0.15)
    big = synth.config4_like(12, 762, min_len=4800, max_len=6200, max_div=0.06)
    pairs = [b.pair(p) for p in range(b.n_pairs)] + [big.pair(p) for p in range(big.n_pairs)]
    bb = synth.from_pairs("packed band", pairs, DNA, 5, 2, 0)
    want = oracle_mod.align_batch(bb.seqs_a, bb.offs_a, bb.seqs_b, bb.offs_b, DNA, 5, 2, 0)
    dev = gpu.to_device(bb)
    # the last case spreads the first round over every lane-width class
    for w0, rounds in ((0, 6), (20, 6), (120, 6), (3, 2), (None, 3)):
        if w0 is None:
            w = _w(torch, rng.integers(0, 520, bb.n_pairs))
        else:
            w = _w(torch, rng.integers(max(0, w0 - 3), w0 + 4, bb.n_pairs))
        res = {}
        for on in (True, False):
            gpu.set_band_packing(on)
            sc, st = gpu.align_batch_band(*dev, DNA, 5, 2, 0, w, max_rounds=rounds)
            res[on] = sc.cpu().numpy()
            _say(f"packed={on} w0~{w0} rounds={rounds}: {st}")
            assert np.array_equal(res[on], want), (on, w0, np.nonzero(res[on] != want)[0][:5])
    gpu.set_band_packing(True)


def test_packed_band_lower_range_harsh_scoring(gpu, oracle_mod):
    """A scheme whose diagonal steps lose score in the shifted frame (sigma
    + 2 beta < 0): banded cells of long pairs fall far below zero, so the
    packed kernel's range proof must also bound them from below and send
    the longest pairs to the 32-bit kernel.  Every score equals the
    oracle's, with the packed kernel on and off."""
    import torch
    rng = np.random.default_rng(780)
    sub = np.full((4, 4), -12, dtype=np.int8)
    np.fill_diagonal(sub, 3)
    alpha, beta = 12, 0
    lens = [300, 900, 1500, 2300, 2900, 3600]
    pairs = []
    for L in lens:
        for rel in (True, False):
            a = rng.integers(0, 4, L).astype(np.uint8)
            if rel:
                sb, _ = synth.mutate(rng, a, np.array([0, L]), [0.08], [0.02], [0.02], 4)
            else:
                sb = rng.integers(0, 4, L + int(rng.integers(-40, 40))).astype(np.uint8)
            pairs.append((a, sb))
    bb = synth.from_pairs("harsh", pairs, sub, alpha, beta, 0)
    want = oracle_mod.align_batch(bb.seqs_a, bb.offs_a, bb.seqs_b, bb.offs_b, sub, alpha, beta, 0)
    dev = gpu.to_device(bb)
    w = _w(torch, np.full(bb.n_pairs, 60))
    for on in (True, False):
        gpu.set_band_packing(on)
        sc, st = gpu.align_batch_band(*dev, sub, alpha, beta, 0, w, max_rounds=4)
        _say(f"harsh scoring packed={on}: {st}")
        assert np.array_equal(sc.cpu().numpy(), want), (on, np.nonzero(sc.cpu().numpy() != want)[0])
    gpu.set_band_packing(True)


def test_wide_band_classes(gpu, oracle_mod):
    """Bands of 1280 and 1536 diagonals (whole-wave lane groups with K = 20
    and 24 registers per lane): pairs of ~3000 residues take the packed
    kernel, pairs of ~10500 (past the packed range proof) the 32-bit one.
    Related pairs at 10-14% (short) or 5-6.5% (long) divergence need more
    than 1024 diagonals, so the wide classes accept what the full DP would
    otherwise compute; unrelated pairs are rejected and fall back.  Every
    score equals the oracle's, with the packed kernel on and off."""
    import torch
    rng = np.random.default_rng(790)
    pairs = []
    for L, divs in ((2900, (0.10, 0.14)), (3100, (0.10, 0.14)), (10400, (0.05, 0.065)), (10600, (0.05, 0.065))):
        for div in divs + (None,):
            a = rng.integers(0, 4, L).astype(np.uint8)
            if div is None:
                sb = rng.integers(0, 4, L + int(rng.integers(-30, 30))).astype(np.uint8)
            else:
                sb, _ = synth.mutate(rng, a, np.array([0, L]), [div / 2], [div / 4], [div / 4], 4)
            pairs.append((a, sb))
    bb = synth.from_pairs("wide bands", pairs, DNA, 5, 2, 0)
    want = oracle_mod.align_batch(bb.seqs_a, bb.offs_a, bb.seqs_b, bb.offs_b, DNA, 5, 2, 0)
    dev = gpu.to_device(bb)
    dn = np.abs(bb.lens_a.astype(np.int64) - bb.lens_b.astype(np.int64))
    for need in (1200, 1500):
        # half-widths whose request needs about `need` diagonals
        w = _w(torch, np.maximum(0, (need - 1 - dn) // 2))
        for on in (True, False):
            gpu.set_band_packing(on)
            sc, st = gpu.align_batch_band(*dev, DNA, 5, 2, 0, w, max_rounds=3)
            _say(f"wide bands need~{need} packed={on}: {st}")
            assert np.array_equal(sc.cpu().numpy(), want), (need, on, np.nonzero(sc.cpu().numpy() != want)[0])
            assert st["accepted"][0] >= 4, st
            if on:
                assert st["band16_cells"] > 0 and st["band_cells"] > st["band16_cells"], st
    gpu.set_band_packing(True)


def test_global_retry_settles_in_round_two(gpu, oracle_mod):
    """A rejected global band retries at the half-width its banded score
    would pass; the retry's band contains the rejected one, so its score is
    at least as high and it passes: every pair is settled (accepted or sent
    to the full DP) by the second round, from any initial width.  Scores
    equal the oracle's, packed kernel on and off."""
    import torch
    b = synth.config4_like(1500, 795, min_len=300, max_len=3000, max_div=0.15)
    want = oracle_mod.align_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, DNA, 5, 2, 0)
    dev = gpu.to_device(b)
    for w0 in (0, 10, 60):
        w = _w(torch, np.full(b.n_pairs, w0))
        for on in (True, False):
            gpu.set_band_packing(on)
            sc, st = gpu.align_batch_band(*dev, DNA, 5, 2, 0, w, max_rounds=6)
            _say(f"retry w0={w0} packed={on}: {st}")
            assert np.array_equal(sc.cpu().numpy(), want), (w0, on, np.nonzero(sc.cpu().numpy() != want)[0][:5])
            assert sum(st["accepted"][2:]) == 0 and len(st["accepted"]) == 2 and st["accepted"][1] > 0, st
    gpu.set_band_packing(True)


# Lane-width classes of the two banded kernels (diagonals).
PACKED_WIDTHS = (80, 96, 112, 128, 160, 192, 224, 256, 320, 384, 448, 512, 640, 768, 896, 1024,
                 1280, 1536)
WIDTHS32 = (64, 128, 192, 256, 384, 512, 768, 1024, 1280, 1536)


def test_raw_packed_band_every_class(gpu, oracle_mod):
    """Raw banded scores of the packed 16-bit kernel against the oracle's DP
    restricted to the diagonals it reports, in every one of its 18 classes:
    per class, pairs of 300-2600 residues with unequal row counts (so the
    two halves of a lane group end on different steps) and requests that
    just fit the class; the 96/192/384/768 and 1280 classes run their
    selector rotation in phases (K = 6, 12, 20).  Pairs of 4.8-6.2 kb in
    the widest classes carry the lowered bias (their upper bound passes
    32768).  With packing off the same requests take the 32-bit kernel;
    both equal the oracle."""
    import torch
    rng = np.random.default_rng(7300)
    pairs, target = [], []
    for W in PACKED_WIDTHS:
        base = synth.config4_like(36, int(rng.integers(1 << 30)), min_len=max(300, (4 * W) // 3 + 40),
                                  max_len=max(900, (4 * W) // 3 + 1400), max_div=0.12)
        for p in range(base.n_pairs):
            pairs.append(base.pair(p))
            target.append(W)
    big = synth.config4_like(10, 7301, min_len=4800, max_len=6200, max_div=0.08)
    for p in range(big.n_pairs):
        pairs.append(big.pair(p))
        target.append(1280 if p % 2 else 1536)
    bb = synth.from_pairs("raw packed", pairs, DNA, 5, 2, 0)
    target = np.asarray(target)
    dn = np.abs(bb.lens_a.astype(np.int64) - bb.lens_b.astype(np.int64))
    keep = dn + 1 <= target
    bb = bb.subset(np.nonzero(keep)[0])
    target, dn = target[keep], dn[keep]
    w = np.maximum(0, (target - 1 - dn) // 2)          # B = dn + 2w + 1 just fits the class
    dev = gpu.to_device(bb)
    L = np.minimum(0, bb.lens_b - bb.lens_a) - w
    U = np.maximum(0, bb.lens_b - bb.lens_a) + w
    for on in (True, False):
        gpu.set_band_packing(on)
        got, lo, hi = gpu.band_scores(*dev, DNA, 5, 2, 0, _w(torch, w))
        got, lo, hi = got.cpu().numpy(), lo.cpu().numpy(), hi.cpu().numpy()
        widths = hi - lo + 1
        _say(f"raw packed={on}: {bb.n_pairs} pairs, widths {sorted(set(widths.tolist()))}")
        assert np.all(lo <= L) and np.all(hi >= U)
        if on:
            assert np.array_equal(widths, target), np.nonzero(widths != target)[0][:5]
        else:
            assert set(widths.tolist()) <= set(WIDTHS32)
        want = oracle_mod.diag_band_batch(bb.seqs_a, bb.offs_a, bb.seqs_b, bb.offs_b, DNA, 5, 2, 0, lo, hi)
        bad = np.nonzero(got.astype(np.int64) != want)[0]
        assert len(bad) == 0, (f"packed={on}: {len(bad)} mismatches, first pair {bad[0]}: gpu {got[bad[0]]} "
                               f"oracle {want[bad[0]]} m={bb.lens_a[bad[0]]} n={bb.lens_b[bad[0]]} "
                               f"lo={lo[bad[0]]} hi={hi[bad[0]]}")
    gpu.set_band_packing(True)


def _widest_packed(m, n):
    """Widest packed class a global pair may take in the rounds (at most
    three quarters of the longer sequence; DNA pairs of these lengths pass
    the range proof)."""
    ok = [W for W in PACKED_WIDTHS if 4 * W <= 3 * max(m, n)]
    return max(ok) if ok else 0


def test_no_fallback_when_first_band_holds_the_path(gpu, oracle_mod):
    """Pairs whose first computed band already holds an optimal path (the
    oracle's score of that band equals the full DP's) and whose
    certificate width fits a class: a rejected band retries at the width
    its score passes, so every such pair is accepted by the second round
    and none falls back to the full DP."""
    import torch
    b = synth.config4_like(1200, 7310, min_len=1200, max_len=3200, max_div=0.08)
    full = oracle_mod.align_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, DNA, 5, 2, 0)
    m = b.lens_a.astype(np.int64)
    n = b.lens_b.astype(np.int64)
    mn, dn = np.minimum(m, n), np.abs(n - m)
    # smallest half-width whose leave bound the full score passes (global)
    num = 2 * (mn - 1) - 2 * 5 - 2 * dn - full
    wcert = np.where(num <= 0, 0, (num + 5) // 6)
    widest = np.array([_widest_packed(int(a), int(c)) for a, c in zip(m, n)])
    gpu.set_band_packing(True)
    dev = gpu.to_device(b)
    for w0 in (0, 10):
        w = np.full(b.n_pairs, w0)
        _, lo, hi = gpu.band_scores(*dev, DNA, 5, 2, 0, _w(torch, w))
        first = oracle_mod.diag_band_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, DNA, 5, 2, 0,
                                           lo.cpu().numpy(), hi.cpu().numpy())
        sel = np.nonzero((first == full) & (dn + 2 * wcert + 1 <= widest))[0]
        assert len(sel) > b.n_pairs // 2
        sub = b.subset(sel)
        sc, st = gpu.align_batch_band(*gpu.to_device(sub), DNA, 5, 2, 0, _w(torch, w[sel]), max_rounds=6)
        _say(f"first band holds the path, w0={w0}: {len(sel)} pairs, {st}")
        assert np.array_equal(sc.cpu().numpy(), full[sel])
        assert st["fallback"] == 0 and sum(st["accepted"][2:]) == 0, st
