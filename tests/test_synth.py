"""Input generators: shapes and reproducibility (no method arithmetic here)."""
import numpy as np

import synth


def test_unique_uniform_keys_exact_count_and_range():
    k = synth.unique_uniform_keys(200000, 5, bits=20)   # forces many repeats, then top-up
    assert len(k) == 200000 and len(np.unique(k)) == 200000
    assert int(k.max()) < (1 << 20)


def test_sample_indices_distinct():
    for n, k in ((10, 10), (1000, 3), (10 ** 6, 5000)):
        idx = synth.sample_indices(n, k, 9)
        assert len(idx) == k and len(np.unique(idx)) == k and idx.min() >= 0 and idx.max() < n


def test_zipf_lengths_range_and_skew():
    l = synth.zipf_lengths(100000, 3, alpha=1.2, lmax=10 ** 6)
    assert l.min() >= 1 and l.max() <= 10 ** 6
    assert 0.15 < np.mean(l == 1) < 0.25          # P(1) = 1/zeta_N(1.2) ~ 0.19


def test_rmat_torch_matches_numpy():
    s1, d1 = synth.rmat_edges(4000, 11, scale=14)
    s2, d2 = synth.rmat_edges_torch(4000, 11, scale=14)
    assert np.array_equal(s1.astype(np.int64), s2.numpy())
    assert np.array_equal(d1.astype(np.int64), d2.numpy())
    assert int(s1.max()) < (1 << 14) and int(d1.max()) < (1 << 14)
    # vertex 0 is the hub of the (a=.5, b=c=.1, d=.3) recursion
    s3, d3 = synth.rmat_edges(200000, 12, scale=10)
    deg = np.bincount(np.concatenate([s3, d3]).astype(np.int64))
    assert deg.argmax() == 0


def test_uniform_keys_at_matches_stream():
    full = synth.uniform_keys(5000, 77, bits=40, offset=123)
    idx = np.array([0, 1, 17, 4999, 2500], dtype=np.int64)
    assert np.array_equal(synth.uniform_keys_at(idx + 123, 77, bits=40), full[idx])


def test_zipf_keys_shape():
    """Zipf(0.99) over 2^34 ranks: keys below 2^34, the two most popular keys
    drawn exactly with their probabilities 1 / zeta and 2^-0.99 / zeta (within
    sampling error), rank frequencies falling, and zeta against a direct sum."""
    n = 400000
    k = synth.zipf_keys(n, 31)
    assert k.dtype == np.uint64 and int(k.max()) < (1 << 34)
    z = synth.zipf_zeta(1 << 34, 0.99)
    f = np.bincount(k[k < 8].astype(np.int64), minlength=8) / n
    for r, p in ((1, 1.0 / z), (2, 2.0 ** -0.99 / z)):
        sd = (p * (1 - p) / n) ** 0.5
        assert abs(f[r - 1] - p) < 5 * sd
    assert all(f[i] > f[i + 1] for i in range(4))
    i = np.arange(1, 3_000_001, dtype=np.float64)
    assert abs(synth.zipf_zeta(3_000_000, 0.99, head=1 << 12) - float(np.sum(i ** -0.99))) < 1e-9
    assert np.array_equal(synth.zipf_keys(100, 31, offset=50), k[50:150])


def test_er_edges_uniform_and_torch_twin():
    import torch
    s, d = synth.er_edges(200000, 61, 1000)
    assert int(s.max()) < 1000 and int(d.max()) < 1000
    counts = np.bincount(s.astype(np.int64), minlength=1000)
    assert abs(counts.mean() - 200) < 1e-9 and counts.std() < 3 * 200 ** 0.5   # about Poisson(200)
    ts, td = synth.er_edges_torch(200000, 61, 1000)
    assert np.array_equal(ts.numpy().astype(np.uint64), s) and np.array_equal(td.numpy().astype(np.uint64), d)
