"""Generator checks: determinism, sizes, the foreign-key property, the key
distributions the workloads promise."""
import numpy as np

import workloads


def test_fk_small_shape_and_fk_property():
    w = workloads.make("fk_small", scale_shift=6)
    assert w.R.shape == (1 << 14, 2) and w.S.shape == (1 << 16, 2)
    assert sorted(w.R[:, 0].tolist()) == list(range(1 << 14))        # a permutation of [0, nR)
    assert np.array_equal(w.S[:, 0], w.R[w.partner.astype(np.int64), 0])
    w2 = workloads.make("fk_small", scale_shift=6)
    assert np.array_equal(w.R, w2.R) and np.array_equal(w.S, w2.S)


def test_fk_uniform_spread_keys_unique_and_wide():
    w = workloads.make("fk_uniform", scale_shift=10)
    k = w.R[:, 0]
    assert len(np.unique(k)) == len(k)
    assert int(k.max()) > (1 << 62) and np.array_equal(w.S[:, 0], k[w.partner.astype(np.int64)])


def test_skewed_zipf_head():
    w = workloads.make("skewed", scale_shift=8)      # |R| = 2^18, |S| = 2^20
    assert len(np.unique(w.R[:, 0])) == len(w.R)
    _, c = np.unique(w.partner, return_counts=True)
    top = c.max() / len(w.S)
    harmonic = np.sum(1.0 / np.arange(1, len(w.R) + 1))
    assert abs(top - 1.0 / harmonic) < 0.01          # Zipf(1): p(rank 1) = 1 / H_N


def test_lognormal_counts():
    w = workloads.make("lognormal", scale_shift=14)
    assert w.R.shape == (1 << 14, 2) and w.S.shape == (1 << 16, 2)
    ks, cs = np.unique(w.S[:, 0], return_counts=True)
    kr = np.unique(w.R[:, 0])
    assert np.array_equal(ks, kr)                    # every distinct R key, and only those
    assert cs.min() >= 1 and cs.max() <= 16


def test_batch_sizes():
    b = workloads.make("batch", scale_shift=6)
    assert len(b) == 4
    for w in b:
        assert len(w.S) % len(w.R) == 0 and 1 <= len(w.S) // len(w.R) <= 8
        assert np.array_equal(w.S[:, 0], w.R[w.partner.astype(np.int64), 0])
