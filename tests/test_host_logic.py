"""Host-side routing helpers of the HIP runtime (compiled for the CPU from
the same header, no GPU): the retry width of a rejected global band against
the oracle's acceptance bound, the packed banded kernel's range proof and
bias, the class ladders and the band routing."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def host(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("host") / "host_logic")
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O1",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2205_07610_amd", "csrc"),
                           os.path.join(HERE, "host_logic.hip"), "-o", exe])

    def run(lines):
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                             check=True).stdout
        return out.strip().splitlines()
    return run


def test_retry_width_is_the_smallest_passing_band(host):
    """band_w_for_score(m, n, S) is the smallest half-width whose band the
    oracle's leave bound lets S pass (equal while the band stays inside the
    matrix, never smaller at its edge)."""
    from oracle import GLOBAL
    from oracle.band import ub_outside
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(400):
        m, n = int(rng.integers(1, 400)), int(rng.integers(1, 400))
        sm = int(rng.integers(1, 6))
        beta = int(rng.integers(0, 4))
        alpha = beta + int(rng.integers(0, 10))
        s = int(rng.integers(-3 * (m + n), sm * min(m, n) + 1))
        cases.append((m, n, s, sm, alpha, beta))
    got = [int(x) for x in host([f"w {m} {n} {s} {sm} {a} {b}" for m, n, s, sm, a, b in cases])]
    for (m, n, s, sm, a, b), w in zip(cases, got):
        wb = 0
        while True:
            ub = ub_outside(m, n, wb, sm, a, b, GLOBAL)
            if ub is None or s >= ub:
                break
            wb += 1
        inside = min(0, n - m) - wb - 1 >= -m and max(0, n - m) + wb + 1 <= n
        if inside:
            assert w == wb, (m, n, s, sm, a, b, w, wb)
        else:
            assert w >= wb, (m, n, s, sm, a, b, w, wb)


def test_packed_range_proof_and_bias(host):
    """A range-proven pair's cells, from -LB to UB, stay inside [1, 65280]
    after its bias; a pair with UB + LB >= 65000 is refused."""
    rng = np.random.default_rng(12)
    cases = []
    for _ in range(500):
        m = int(rng.integers(1, 20000))
        n = m + int(rng.integers(0, 3000))
        W = int(rng.choice([80, 320, 1024, 1536]))
        sp, dr = int(rng.integers(0, 12)), int(rng.integers(0, 14))
        b = int(rng.integers(0, 4))
        a = b + int(rng.integers(0, 12))
        cases.append((m, n, W, sp, dr, a, b))
    got = host([f"r {m} {n} {W} {sp} {dr} {a} {b}" for m, n, W, sp, dr, a, b in cases])
    seen = {0: 0, 1: 0}
    for (m, n, W, sp, dr, a, b), line in zip(cases, got):
        ok, bias, ub, lb = (int(x) for x in line.split())
        assert ub == sp * min(m, n) + b * (m + n + W) + a + 2 * b + 256
        assert lb == dr * min(m, n) + 3 * (a - b) + 256
        assert ok == int(lb < 32000 and ub + lb < 65000)
        seen[ok] += 1
        if ok:
            assert bias - lb >= 1 and ub + bias <= 65280 and bias <= 32768
    assert seen[0] > 20 and seen[1] > 20


def test_class_ladders_and_routing(host):
    """Class widths grow by at most 1.25x (packed) and 1.5x (32-bit, from 128
    on); a routed band holds the request and obeys the worth and range
    rules."""
    w16, w32 = ([int(x) for x in line.split()] for line in host(["c"]))
    assert w16[0] == 80 and w16[-1] == 1536 and w32[-1] == 1536
    for ws, r in ((w16, 1.25), (w32[1:], 1.5)):
        assert all(b > a and b <= r * a for a, b in zip(ws, ws[1:]))
    assert w32[:2] == [64, 128]
    rng = np.random.default_rng(13)
    cases = []
    for _ in range(400):
        m = int(rng.integers(50, 6000))
        n = m + int(rng.integers(0, 300))
        w = int(rng.integers(0, 900))
        cases.append((m, n, w, 2, 0, 5, 2))
    got = host([f"p {m} {n} {w} {sp} {dr} {a} {b}" for m, n, w, sp, dr, a, b in cases])
    routed = 0
    for (m, n, w, sp, dr, a, b), line in zip(cases, got):
        packed, c, W = (int(x) for x in line.split())
        need = n - m + 2 * w + 1
        if c < 0:
            continue
        routed += 1
        assert W >= need
        if packed:
            ub = sp * m + b * (m + n + W) + a + 2 * b + 256
            assert 4 * W <= 3 * n and ub + 3 * (a - b) + 256 < 65000
            assert W == min(x for x in w16 if x >= need)
        else:
            assert 2 * W < n
    assert routed > 100


def test_fp8_profile_codes(host):
    """The packed kernel's FP16 cells read profile bytes as FP8 codes.  E4M3
    codes of 0..16 decode (sign 0, 4-bit exponent with bias 7, 3-bit
    mantissa) to the integer itself; E5M2 codes shifted into the upper byte
    of a 16-bit word are the IEEE half of the integer (decoded by numpy),
    for exactly the integers the exactness test admits."""
    got = [tuple(int(x) for x in line.split()) for line in host([f"f {v}" for v in range(17)])]
    for v, (e4, e5, ex) in enumerate(got):
        if v == 0:
            assert e4 == 0 and e5 == 0
        else:
            e, m = e4 >> 3, e4 & 7
            assert e4 < 128 and 2.0 ** (e - 7) * (1 + m / 8) == v, (v, e4)
        half = float(np.array([e5 << 8], dtype=np.uint16).view(np.float16)[0])
        want_exact = float(np.float16(v)) == v and (np.array([np.float16(v)]).view(np.uint16)[0] & 0xFF) == 0
        assert bool(ex) == bool(want_exact), (v, ex)
        if ex:
            assert half == v, (v, e5, half)
    assert [v for v, g in enumerate(got) if g[2]] == [0, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16]
