"""Pins for the learned-band parts of the oracle: the per-pair k-mer features,
the band network (float64 with bfloat16 rounding points), its loss, its
optimiser and the band label.

Features are pinned by hand-built pairs whose diagonal histogram can be
worked out on paper (a shifted copy, a trimmed copy, duplicated k-mers, the
position cap and the last bin).  The network is pinned by central finite
differences (gradients), by torch's own bfloat16 conversion and float64
matrix products (rounding points), and by torch.optim.Adam (optimiser).
"""
import collections
import math

import numpy as np
import pytest
import torch

from oracle import GLOBAL, SEMIGLOBAL
from oracle import band, features as F, mlp

DNA = np.full((4, 4), -3, dtype=np.int8)
np.fill_diagonal(DNA, 2)


def _distinct_kmers(x):
    codes = F.kmer_codes(x)
    return len(set(codes)) == len(codes)


def _seqs_with_distinct_kmers(seed, *lens):
    for s in range(seed, seed + 10_000):
        r = np.random.default_rng(s)
        parts = [r.integers(0, 4, n).tolist() for n in lens]
        if _distinct_kmers(sum(parts, [])):
            return parts
    raise AssertionError("no seed found")


def test_kmer_code_definition():
    # ACGTACG -> 0,1,2,3,0,1,2 in base 4, most significant first
    assert F.kmer_codes([0, 1, 2, 3, 0, 1, 2]) == [0 * 4**6 + 1 * 4**5 + 2 * 4**4 + 3 * 4**3
                                                   + 0 * 4**2 + 1 * 4 + 2]
    assert F.kmer_codes([3] * 8) == [4**7 - 1, 4**7 - 1]
    assert F.kmer_codes([1] * 6) == []


def test_features_shifted_copy():
    """B = X + A, |X| = 10, m = 20: the k-mer at i sits at j = i + 10 and
    the expected diagonal is trunc(10 i / 20) = i // 2, so delta = 10 - i//2:
    10,10,9,9,8,8,7,7 (bin 15 + 3) and 6,6,5,5,4,4 (bin 15 + 2)."""
    x, a = _seqs_with_distinct_kmers(0, 10, 20)
    f = F.pair_features(a, x + a)
    want = np.zeros(32)
    want[18], want[17] = 8 / 14, 6 / 14
    want[30] = math.log2(11) / 16
    want[31] = 14 / 14
    np.testing.assert_allclose(f, want.astype(np.float32), rtol=0, atol=0)


def test_features_trimmed_copy_truncates_toward_zero():
    """B = A[10:], m = 30, n = 20: k-mers at i = 10..23 sit at j = i - 10 and
    the expected diagonal is trunc(-10 i / 30) = -(i // 3) (truncation toward
    zero; floor division would shift half of them), so delta = -10 + i//3:
    -7 x2 (bin 14 - 3), -6 x3, -5 x3, -4 x3, -3 x3 (bin 14 - 2)."""
    (a,) = _seqs_with_distinct_kmers(100, 30)
    f = F.pair_features(a, a[10:])
    want = np.zeros(32)
    want[11], want[12] = 2 / 14, 12 / 14
    want[30] = math.log2(11) / 16
    want[31] = 14 / 24
    np.testing.assert_allclose(f, want.astype(np.float32), rtol=0, atol=0)


def test_features_duplicated_kmers_are_not_used():
    (a,) = _seqs_with_distinct_kmers(200, 20)
    f = F.pair_features(a, a + a)       # every k-mer of A occurs twice in B
    want = np.zeros(32)
    want[30] = math.log2(21) / 16
    np.testing.assert_array_equal(f, want.astype(np.float32))


def test_features_short_and_empty():
    for a, b in (([], []), ([0, 1, 2], [0, 1, 2]), ([0] * 6, [0] * 100), ([1] * 50, [])):
        f = F.pair_features(a, b)
        assert f[:30].sum() == 0 and f[31] == 0
        assert f[30] == np.float32(math.log2(1 + abs(len(a) - len(b))) / 16)


@pytest.mark.parametrize("j,usable", [(65534, True), (65535, False)])
def test_features_position_cap_and_last_bin(j, usable):
    """A = GGGGGGG (one k-mer, i = 0); B is ACAC... with GGGGGGG planted at
    j.  delta = j, floor(log2(1 + j)) = 15 is clamped to 14 (bin 29); a
    k-mer starting at 65535 or later is not usable."""
    b = ([0, 1] * 40_000)[:70_000]
    b[j:j + 7] = [2] * 7
    f = F.pair_features([2] * 7, b)
    if usable:
        assert f[29] == 1.0 and f[31] == 1.0 and f[:29].sum() == 0
    else:
        assert f[:30].sum() == 0 and f[31] == 0


def test_features_identical_sequences():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 4, 500).tolist()
    counts = collections.Counter(F.kmer_codes(a))
    unique = sum(1 for c in F.kmer_codes(a) if counts[c] == 1)
    f = F.pair_features(a, a)
    assert f[15] == 1.0 and f[:15].sum() == 0 and f[16:30].sum() == 0
    assert f[31] == np.float32(unique / (500 - 6))
    assert f[30] == 0


def test_features_histogram_sums_to_one():
    rng = np.random.default_rng(8)
    for _ in range(20):
        a = rng.integers(0, 4, int(rng.integers(20, 300))).tolist()
        b = list(a)
        for _k in range(int(rng.integers(0, 10))):
            p = int(rng.integers(0, len(b)))
            if rng.random() < 0.5:
                del b[p]
            else:
                b.insert(p, int(rng.integers(0, 4)))
        f = F.pair_features(a, b)
        if f[31] > 0:
            assert abs(float(f[:30].sum()) - 1.0) < 1e-6


# ---------------------------------------------------------------- network

def test_bf16_rounding_points():
    one = 1.0
    # bfloat16 keeps 7 fraction bits: spacing 2^-7 at 1
    assert mlp.bf16(one + 2**-8)[()] == 1.0                 # tie -> even (1.0)
    assert mlp.bf16(one + 3 * 2**-8)[()] == one + 2**-6     # tie -> even (1 + 2^-6)
    assert mlp.bf16(one + 2**-8 + 2**-20)[()] == one + 2**-7  # above the tie
    assert mlp.bf16(-(one + 2**-8))[()] == -1.0
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(20_000) * np.exp(rng.uniform(-20, 20, 20_000))).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), want)


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(rng)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape).astype(np.float32)
    return p


def test_forward_matches_torch_with_bf16_casts():
    p = _rand_params(4)
    x = np.random.default_rng(5).uniform(0, 1, (64, 32)).astype(np.float32)
    y, _ = mlp.forward(p, x)

    def r(a):
        return torch.as_tensor(a).to(torch.float32).to(torch.bfloat16).to(torch.float64)
    T = {k: torch.as_tensor(v, dtype=torch.float64) for k, v in p.items()}
    h = torch.relu(r(x) @ r(p["w1"]) + T["b1"])
    h = torch.relu(r(h) @ r(p["w2"]) + T["b2"])
    want = r(h) @ r(p["w3"]) + T["b3"][0]
    np.testing.assert_allclose(y, want.numpy(), rtol=1e-12, atol=1e-12)


def test_backward_matches_finite_differences():
    p = {k: v.astype(np.float64) for k, v in _rand_params(6).items()}
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 1, (8, 32))
    gy = rng.standard_normal(8)

    def obj(pp):
        return float(np.dot(gy, mlp.forward(pp, x, round_=False)[0]))

    _, cache = mlp.forward(p, x, round_=False)
    g = mlp.backward(cache, gy, round_=False)
    h = 1e-6
    for k in mlp.PARAM_NAMES:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(flat.size, 40), replace=False)
        for i in idx:
            save = flat[i]
            flat[i] = save + h
            up = obj(p)
            flat[i] = save - h
            dn = obj(p)
            flat[i] = save
            num = (up - dn) / (2 * h)
            assert abs(num - g[k].reshape(-1)[i]) <= 1e-6 * (1 + abs(num)), (k, i)


def test_pinball_and_its_derivative():
    tau = 0.85
    y = np.array([1.0, 3.0, 2.0])
    t = np.array([2.0, 1.0, 2.0])
    # r = 1 -> tau*1; r = -2 -> (tau-1)*(-2) = 0.3; r = 0 -> 0
    assert mlp.pinball(y, t, tau) == pytest.approx((0.85 + 0.3 + 0) / 3, abs=1e-15)
    g = mlp.dloss_dy(y, t, tau)
    np.testing.assert_allclose(g, [-0.85 / 3, 0.15 / 3, 0.0])
    rng = np.random.default_rng(9)
    y = rng.standard_normal(50)
    t = rng.standard_normal(50)
    g = mlp.dloss_dy(y, t, tau)
    for i in range(50):
        e = np.zeros(50)
        e[i] = 1e-7
        num = (mlp.pinball(y + e, t, tau) - mlp.pinball(y - e, t, tau)) / 2e-7
        assert abs(num - g[i]) < 1e-6


def test_adam_matches_torch():
    p = _rand_params(10)
    rng = np.random.default_rng(11)
    tp = {k: torch.tensor(v.astype(np.float64), requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp[k] for k in mlp.PARAM_NAMES), lr=3e-3, betas=(0.9, 0.999),
                           eps=1e-8)
    cur = {k: v.astype(np.float64) for k, v in p.items()}
    state = {}
    for t in range(1, 4):
        grads = {k: rng.standard_normal(v.shape) for k, v in p.items()}
        cur, state = mlp.adam_step(cur, grads, state, t, lr=3e-3)
        for k in mlp.PARAM_NAMES:
            tp[k].grad = torch.tensor(grads[k])
        opt.step()
        for k in mlp.PARAM_NAMES:
            np.testing.assert_allclose(cur[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)


def test_adam_first_step_closed_form():
    # t = 1: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    g = {k: np.full(np.shape(v), 0.5) for k, v in _rand_params(12).items()}
    p0 = {k: np.zeros(np.shape(v)) for k, v in g.items()}
    p1, _ = mlp.adam_step(p0, g, {}, 1, lr=0.01)
    for k in mlp.PARAM_NAMES:
        np.testing.assert_allclose(p1[k], -0.01 * 0.5 / (0.5 + 1e-8))


def test_predict_width():
    w = np.arange(0, 2000)
    # w + 1 >= 2^y: just below log2(w + 1) gives w, just above gives w + 1
    # (exactly at the boundary the result depends on the last bit of exp2)
    np.testing.assert_array_equal(mlp.predict_width(np.log2(w + 1.0) - 1e-9), w)
    np.testing.assert_array_equal(mlp.predict_width(np.log2(w + 1.0) + 1e-9), w + 1)
    assert mlp.predict_width(np.array([-3.0]))[0] == 0


# ---------------------------------------------------------------- label

def test_band_label(oracle_mod):
    rng = np.random.default_rng(13)
    for _ in range(20):
        a = rng.integers(0, 4, int(rng.integers(30, 200))).tolist()
        b = list(a)
        for _k in range(int(rng.integers(0, 12))):
            p = int(rng.integers(0, len(b)))
            if rng.random() < 0.5:
                del b[p]
            else:
                b.insert(p, int(rng.integers(0, 4)))
        for md in (GLOBAL, SEMIGLOBAL):
            wa = band.accepted_width(a, b, DNA, 5, 2, md)
            assert band.band_label(a, b, DNA, 5, 2, md) == wa
            # a narrow limit turns every label above it into the sentinel
            cap = (31 - abs(len(a) - len(b))) // 2
            lab = band.band_label(a, b, DNA, 5, 2, md, max_band=32)
            assert lab == (wa if 0 <= cap and wa <= cap else 32)
    # identical sequences: the zero-width band already proves the score
    a = rng.integers(0, 4, 300).tolist()
    assert band.band_label(a, a, DNA, 5, 2, GLOBAL) == 0
    # no band fits a length difference of 1024 or more
    assert band.band_label([0] * 10, [0] * 1100, DNA, 5, 2, GLOBAL) == band.MAX_BAND
