"""FP16 cells of the packed full-DP kernel (section 3.2: two alignments in
one register of two half-precision values).  Every score equals the
oracle's, with the FP16 kernel forced for every call that admits it and in
the automatic mode, for FP8 E5M2 and E4M3 profile bytes, in every mode; the
pairs that the FP16 range bound refuses take the 32-bit kernels; a group's
partner running many rows past the other's end stays in range; local
maxima at and around the FP16 re-run threshold are re-run exactly."""
import sys

import numpy as np
import pytest

from paper_2205_07610_amd import synth

pytestmark = pytest.mark.gpu

DNA = synth.dna_subst()
# match 1, mismatch -1, alpha 3, beta 1: sigma + bias and the padding values
# are exact in E5M2 in every mode
SMALL = synth.dna_subst(1, -1)


def _say(msg):
    print(f"[half] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_07610_amd import binding
    binding.lib()
    prev = binding.set_half_cells(2)
    yield binding
    binding.set_half_cells(prev)


def _run(gpu, oracle_mod, b, label, half, cell_type=None, limit=None):
    prev = gpu.set_half_cells(half)
    prev_lim = gpu.set_i16_limit(limit) if limit is not None else None
    prev_t = gpu.enable_timing(True)
    try:
        got = gpu.align(b)
        t = gpu.last_timing()
    finally:
        gpu.enable_timing(prev_t)
        gpu.set_half_cells(prev)
        if prev_lim is not None:
            gpu.set_i16_limit(prev_lim)
    _say(f"{label}: {b.n_pairs} pairs, mode {b.mode}, half {half}: packed {t['pairs_full16']} pairs "
         f"(cell type {t['full16_cell_type']}), re-run {t['pairs_rerun32']}, 32-bit {t['pairs_full32']}")
    want = oracle_mod.align_batch(b.seqs_a, b.offs_a, b.seqs_b, b.offs_b, b.subst, b.alpha, b.beta, b.mode)
    bad = np.nonzero(got.astype(np.int64) != want)[0]
    if len(bad):
        p = int(bad[0])
        raise AssertionError(f"{label}: {len(bad)} mismatches; pair {p}: gpu {got[p]} oracle {want[p]} "
                             f"(m={b.lens_a[p]}, n={b.lens_b[p]})")
    if cell_type is not None:
        assert t["pairs_full16"] > 0, f"{label}: no pair took the packed kernel"
        assert t["full16_cell_type"] == cell_type, (label, t["full16_cell_type"], cell_type)
    return t


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_small_pairs_forced(gpu, oracle_mod, mode):
    """Pairs of 0..300 residues, empty ones included: DNA scoring (E4M3
    bytes in global and semi-global, where sigma + alpha + beta = 9, E5M2 in
    local) and the match-1 scheme (E5M2 everywhere)."""
    rng = np.random.default_rng(1200 + mode)
    sa, oa, sb, ob = synth.random_small(rng, 3000, 300)
    b = synth.Batch("small", sa, oa, sb, ob, DNA, 5, 2, mode)
    _run(gpu, oracle_mod, b, "dna", 1, cell_type=2 if mode == 2 else 1)
    b = synth.Batch("small", sa, oa, sb, ob, SMALL, 3, 1, mode)
    _run(gpu, oracle_mod, b, "match-1", 1, cell_type=2)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_unequal_partners(gpu, oracle_mod, mode):
    """Groups pair a one-row pair with one of up to the FP16 row bound (the
    short half runs far past its end) and columns from 1 to 256."""
    rng = np.random.default_rng(1210 + mode)
    pairs = []
    for k in range(1200):
        m = int(rng.integers(1, 4)) if k % 2 else int(rng.integers(150, 240))
        n = int(rng.integers(1, 257))
        a = rng.integers(0, 4, size=m).astype(np.uint8)
        if rng.random() < 0.5 and m > 3:
            s, _ = synth.mutate(rng, a, np.array([0, m]), 0.05, 0.02, 0.02, 4)
            s = s[:n] if len(s) >= n else np.concatenate([s, rng.integers(0, 4, n - len(s)).astype(np.uint8)])
        else:
            s = rng.integers(0, 4, size=n).astype(np.uint8)
        pairs.append((a, s))
    b = synth.from_pairs("partners", pairs, SMALL, 3, 1, mode)
    _run(gpu, oracle_mod, b, "partners", 1, cell_type=2)


@pytest.mark.parametrize("mode", [0, 1])
def test_range_bound_routes_long_rows_to_32bit(gpu, oracle_mod, mode):
    """Global and semi-global pairs past the FP16 row bound (600 rows
    against 200..256 columns, which the routing keeps in that orientation)
    take the 32-bit kernels under FP16 cells and the packed kernel under
    int16 cells; pairs under the bound take the packed kernel either way."""
    rng = np.random.default_rng(1220 + mode)
    pairs = []
    for k in range(600):
        m = 600 if k % 3 == 0 else int(rng.integers(50, 200))
        n = int(rng.integers(200, 257)) if k % 3 == 0 else int(rng.integers(100, 200))
        pairs.append((rng.integers(0, 4, size=m).astype(np.uint8), rng.integers(0, 4, size=n).astype(np.uint8)))
    b = synth.from_pairs("bound", pairs, DNA, 5, 2, mode)
    t = _run(gpu, oracle_mod, b, "bound", 1, cell_type=1)
    assert t["pairs_full16"] < b.n_pairs
    t16 = _run(gpu, oracle_mod, b, "bound int16", 0, cell_type=0)
    assert t16["pairs_full16"] > t["pairs_full16"]


def test_local_threshold(gpu, oracle_mod):
    """Match 8, mismatch -8, alpha 8, beta 1: bytes 16, 0 and 8 (E5M2).  A
    pair of identical sequences of k residues scores 8k: 247 residues
    (1976) stay below the 1984 threshold, 248 (1984) and 256 (2048) reach
    it and are re-run with 32-bit cells; mutated copies around them too."""
    sub = synth.dna_subst(8, -8)
    rng = np.random.default_rng(1230)
    pairs = []
    for k in (240, 246, 247, 248, 249, 255, 256):
        a = rng.integers(0, 4, size=k).astype(np.uint8)
        pairs.append((a, a.copy()))
        s, _ = synth.mutate(rng, a, np.array([0, k]), 0.01, 0.005, 0.005, 4)
        pairs.append((a, s[:256].astype(np.uint8)))
    for _ in range(200):
        k = int(rng.integers(1, 257))
        a = rng.integers(0, 4, size=k).astype(np.uint8)
        pairs.append((a, rng.integers(0, 4, size=int(rng.integers(1, 257))).astype(np.uint8)))
    b = synth.from_pairs("threshold", pairs, sub, 8, 1, 2)
    t = _run(gpu, oracle_mod, b, "threshold", 1, cell_type=2)
    assert t["pairs_rerun32"] >= 3
    # the automatic mode keeps int16 cells here: the maxima could reach it
    _run(gpu, oracle_mod, b, "threshold auto", 2, cell_type=0)


def test_forced_rerun_and_automatic(gpu, oracle_mod):
    """A lowered threshold from the host sends most FP16 local pairs to the
    32-bit re-run; the automatic mode picks FP16 E5M2 cells for the local
    reads workload's scoring and int16 for the global one."""
    c1 = synth.config1(n_pairs=6000)
    t = _run(gpu, oracle_mod, c1, "c1 forced re-run", 1, cell_type=2, limit=100)
    assert t["pairs_rerun32"] > 0
    _run(gpu, oracle_mod, c1, "c1 auto", 2, cell_type=2)
    _run(gpu, oracle_mod, synth.config0(), "c0 auto", 2, cell_type=0)
    _run(gpu, oracle_mod, synth.config0(), "c0 forced", 1, cell_type=1)


def test_plan_replays_half_cells(gpu, oracle_mod):
    """A plan made under FP16 cells replays to the oracle's scores."""
    import torch
    c1 = synth.config1(n_pairs=3000, seed=1240)
    want = oracle_mod.align_batch(c1.seqs_a, c1.offs_a, c1.seqs_b, c1.offs_b, c1.subst, c1.alpha, c1.beta,
                                  c1.mode)
    prev = gpu.set_half_cells(1)
    try:
        plan = gpu.Plan(*gpu.to_device(c1), c1.subst, c1.alpha, c1.beta, c1.mode)
    finally:
        gpu.set_half_cells(prev)
    for r in range(3):
        got = plan.run().cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got.astype(np.int64), want), f"replay {r}"
    plan.close()
