"""Per-pair features of the band network -- TEST INFRASTRUCTURE ONLY.

Definition (the learned-band extension; the paper has no band):  for a pair
with A of length m (rows) and B of length n (columns), residues 0..3,

* a 7-mer code at position p of a sequence is sum_t x[p+t] * 4^(6-t);
* a 7-mer of B is usable when it occurs exactly once among B's 7-mers that
  start before position 65535;
* for every 7-mer of A at position i whose code is a usable 7-mer of B at
  position j, the deviation from the expected diagonal is
      delta = (j - i) - trunc(i * (n - m) / m)     (C truncation toward 0),
  and it falls into one of 30 signed log bins:
      b = min(14, floor(log2(1 + |delta|))),  bin = 15 + b if delta >= 0
      else 14 - b;
* features 0..29: bin counts divided by max(1, matches); feature 30:
  log2(1 + |n - m|) / 16; feature 31: matches / max(1, m - 6).

Written with plain Python loops over dictionaries so that it can be read
against the definition; it is pinned by hand-built pairs in
tests/test_oracle_learned.py.
"""
from __future__ import annotations

import math

import numpy as np

K = 7
N_FEATURES = 32
MAX_POS = 65535


def kmer_codes(x) -> list[int]:
    x = [int(v) for v in x]
    out = []
    for p in range(len(x) - K + 1):
        c = 0
        for t in range(K):
            c = c * 4 + x[p + t]
        out.append(c)
    return out


def trunc_div(a: int, b: int) -> int:
    q = abs(a) // abs(b)
    return q if (a >= 0) == (b > 0) else -q


def pair_features(a, b) -> np.ndarray:
    m, n = len(a), len(b)
    occ: dict[int, list[int]] = {}
    for j, c in enumerate(kmer_codes(b)):
        if j >= MAX_POS:
            break
        occ.setdefault(c, []).append(j)
    hist = [0] * 30
    matches = 0
    for i, c in enumerate(kmer_codes(a)):
        pos = occ.get(c)
        if pos is None or len(pos) != 1:
            continue
        j = pos[0]
        delta = (j - i) - (trunc_div(i * (n - m), m) if m > 0 else 0)
        b_ = min(14, int(math.floor(math.log2(1 + abs(delta)))))
        hist[15 + b_ if delta >= 0 else 14 - b_] += 1
        matches += 1
    f = np.zeros(N_FEATURES, dtype=np.float64)
    for k in range(30):
        f[k] = hist[k] / max(1, matches)
    f[30] = math.log2(1 + abs(n - m)) / 16.0
    f[31] = matches / max(1, m - (K - 1))
    return f.astype(np.float32)


def batch_features(batch) -> np.ndarray:
    return np.stack([pair_features(*batch.pair(p)) for p in range(batch.n_pairs)]) \
        if batch.n_pairs else np.zeros((0, N_FEATURES), np.float32)
