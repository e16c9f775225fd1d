"""as_align_batch_noalloc (the entry point for callers that cannot allocate)
against as_align_batch: the same scores, bit for bit, on two calls in a row
whose second input is smaller, in every mode and through every full-DP route
(packed 16-bit, 32-bit stripes, 32-bit and packed wavefronts, the 32-bit
re-run of saturated pairs); batches too large for the scratch array are
refused with AS_ERR_SCRATCH."""
import sys

import numpy as np
import pytest

from paper_2205_07610_amd import synth

pytestmark = pytest.mark.gpu

DNA = synth.dna_subst()
AS_ERR_SCRATCH = -8


def _say(msg):
    print(f"[noalloc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_07610_amd import binding
    binding.lib()
    return binding


def _mixed(seed, n_short, n_mid, long_shapes, mode):
    """Short pairs (packed full DP), medium pairs of several stripes, long
    pairs for the wavefronts, and empty sequences."""
    rng = np.random.default_rng(seed)
    pairs = []
    for p in range(n_short):
        m = int(rng.integers(1, 250))
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        b, _ = synth.mutate(rng, a, np.array([0, m]), 0.05, 0.02, 0.02, 4)
        pairs.append((a, b))
    for p in range(n_mid):
        m, n = (int(x) for x in rng.integers(300, 1800, size=2))
        pairs.append((rng.integers(0, 4, size=m).astype(np.uint8),
                      rng.integers(0, 4, size=n).astype(np.uint8)))
    for m, n in long_shapes:
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        b, _ = synth.mutate(rng, a, np.array([0, m]), 0.05, 0.02, 0.02, 4)
        b = b[:n] if len(b) >= n else np.concatenate([b, rng.integers(0, 4, n - len(b)).astype(np.uint8)])
        pairs.append((a, b))
    pairs.append((np.zeros(0, np.uint8), rng.integers(0, 4, size=7).astype(np.uint8)))
    pairs.append((np.zeros(0, np.uint8), np.zeros(0, np.uint8)))
    order = rng.permutation(len(pairs))
    return synth.from_pairs("noalloc", [pairs[i] for i in order], DNA, 5, 2, mode)


def _both(gpu, batch, label):
    import torch
    dev = gpu.to_device(batch, "cuda:0")
    want = gpu.align_batch(*dev, batch.subst, batch.alpha, batch.beta, batch.mode).cpu().numpy()
    # poison the output so a pair the call never writes cannot pass
    out = torch.full((batch.n_pairs,), -(1 << 30), dtype=torch.int32, device="cuda:0")
    got = gpu.align_batch_noalloc(*dev, batch.subst, batch.alpha, batch.beta, batch.mode, out)
    got = got.cpu().numpy()
    bad = np.nonzero(got != want)[0]
    _say(f"{label}: {batch.n_pairs} pairs, {batch.cells():.3g} cells, {len(bad)} mismatches")
    assert len(bad) == 0, (f"{label}: pair {bad[0]}: noalloc {got[bad[0]]} vs as_align_batch "
                           f"{want[bad[0]]}")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_noalloc_matches_align_batch(gpu, mode):
    big = _mixed(7000 + mode, 600, 40, [(2100, 3000), (4097, 2500), (3000, 3300)], mode)
    small = _mixed(7100 + mode, 90, 5, [(2048, 1100)], mode)
    gpu.enable_timing(True)
    try:
        _both(gpu, big, f"mode {mode}, first call")
        tm = gpu.last_timing()  # counts of the no-allocation call: the routes it took
    finally:
        gpu.enable_timing(False)
    assert tm["pairs_full16"] > 0 and tm["pairs_full32"] > 0
    assert tm["pairs_long"] + tm["pairs_long16"] > 0
    _both(gpu, small, f"mode {mode}, second call (smaller)")


def test_noalloc_rerun_of_saturated_pairs(gpu):
    """Local pairs forced through the 32-bit re-run (saturation threshold
    lowered from the host), then a smaller batch."""
    prev = gpu.set_i16_limit(40)
    try:
        _both(gpu, _mixed(7200, 400, 10, [], 2), "local, forced re-run")
        _both(gpu, _mixed(7201, 50, 0, [], 2), "local, forced re-run, smaller")
    finally:
        gpu.set_i16_limit(prev)


def test_noalloc_refuses_what_does_not_fit(gpu):
    import torch
    # the work lists alone exceed the array
    n = 400_000
    oa = torch.arange(n + 1, dtype=torch.int64, device="cuda:0")
    seqs = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    out = torch.empty(n, dtype=torch.int32, device="cuda:0")
    with pytest.raises(gpu.AlignError) as e:
        gpu.align_batch_noalloc(seqs, oa, seqs, oa, DNA, 5, 2, 2, out)
    assert e.value.code == AS_ERR_SCRATCH
    # one long local pair whose wavefront boundary columns exceed what is left
    m = 120_000
    rng = np.random.default_rng(7300)
    b = synth.from_pairs("huge", [(rng.integers(0, 4, size=m).astype(np.uint8),
                                   rng.integers(0, 4, size=m).astype(np.uint8))], DNA, 5, 2, 2)
    dev = gpu.to_device(b, "cuda:0")
    out = torch.empty(1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(gpu.AlignError) as e:
        gpu.align_batch_noalloc(*dev, b.subst, b.alpha, b.beta, b.mode, out)
    assert e.value.code == AS_ERR_SCRATCH
    # and the next call that fits still matches
    _both(gpu, _mixed(7301, 100, 4, [(2100, 2200)], 0), "after refusals")
