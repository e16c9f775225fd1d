"""The seeded input generators: determinism, independence of the thread
count, and the statistics of the mutation model (C generator)."""
import numpy as np

from paper_2205_07610_amd import synth


def test_native_generator_is_deterministic_and_thread_independent():
    lens = np.random.default_rng(1).integers(0, 3000, 300)
    a1, o1 = synth.native_csr(7, lens, 4, nthreads=1)
    a8, o8 = synth.native_csr(7, lens, 4, nthreads=8)
    assert np.array_equal(a1, a8) and np.array_equal(o1, o8)
    assert a1.max() <= 3 and abs(np.bincount(a1, minlength=4) / len(a1) - 0.25).max() < 0.01
    b1, ob1 = synth.native_mutate(9, a1, o1, 0.05, 0.02, 0.02, 4, nthreads=1)
    b8, ob8 = synth.native_mutate(9, a1, o1, 0.05, 0.02, 0.02, 4, nthreads=8)
    assert np.array_equal(b1, b8) and np.array_equal(ob1, ob8)
    p20, _ = synth.native_csr(3, [5000], 20)
    assert p20.max() == 19 and p20.min() == 0


def test_native_mutation_statistics():
    lens = np.full(200, 5000)
    a, oa = synth.native_csr(11, lens, 4)
    # substitutions only: same lengths, about p_sub of the residues differ, never equal-by-substitution
    b, ob = synth.native_mutate(12, a, oa, 0.1, 0.0, 0.0, 4)
    assert np.array_equal(oa, ob)
    frac = np.mean(a != b)
    assert abs(frac - 0.1) < 0.005
    # insertions only: mean growth p_ins * E[L] = p_ins * 2 per residue
    b, ob = synth.native_mutate(13, a, oa, 0.0, 0.03, 0.0, 4)
    growth = (ob[-1] - oa[-1]) / oa[-1]
    assert abs(growth - 0.06) < 0.004
    # deletions only: shrink close to p_del * 2 (overlaps make it slightly less)
    b, ob = synth.native_mutate(14, a, oa, 0.0, 0.0, 0.03, 4)
    shrink = (oa[-1] - ob[-1]) / oa[-1]
    assert 0.05 < shrink < 0.062
    # zero divergence copies
    b, ob = synth.native_mutate(15, a, oa, 0.0, 0.0, 0.0, 4)
    assert np.array_equal(a, b)


def test_config4_law_shapes():
    b = synth.config4_like(2000, 5, min_len=1000, max_len=5000)
    la, lb = b.lens_a, b.lens_b
    assert la.min() >= 1000 and la.max() <= 5000
    # divergence U[0, 0.1] with half indels: |n - m| stays small
    assert np.mean(np.abs(lb - la)) < 0.05 * np.mean(la)
    again = synth.config4_like(2000, 5, min_len=1000, max_len=5000)
    assert np.array_equal(b.seqs_b, again.seqs_b)
