"""Parity at the benchmarked size: a CPMA of 1e8 distinct uniform 40-bit keys,
built and updated as the insert benchmark does (same seeds, device-resident
batches of 1e7 keys, the same launch configuration), then a delete batch of
1e7 present keys.  The CPU oracle is plain C and fast enough at this size to
check everything exactly: n_added / n_removed, the whole exported image through
the structure checker (every key, head, used count, zero fill and node bound),
range sums on sampled short and long ranges, and membership of sampled present
and absent keys."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

N0 = 10 ** 8
K = 10 ** 7


@pytest.fixture(scope="module")
def cp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_05055_amd as p
    p.lib()
    return p


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def check(c, expect, orc):
    b, u, h = c.export()
    code, msg = orc.check_image(b, u, h, c.geometry()[1], expect)
    assert code == 0, msg
    assert c.size() == len(expect)


def test_headline_size_insert_range_delete_exact(cp, orc):
    seed = synth.SEED_BASE + 2
    # base set: exactly N0 distinct keys, topped up from the same stream
    keys = synth.uniform_keys(N0, seed)
    c = cp.CPMA(to_dev(keys))
    parts, off = [keys], N0
    while c.size() < N0:
        more = synth.uniform_keys(N0 - c.size(), seed, offset=off)
        off += len(more)
        c.insert_batch(to_dev(more))
        parts.append(more)
    S = orc.build_set(np.concatenate(parts))
    del keys, parts
    assert len(S) == N0 == c.size()

    # two insert batches of 1e7, as the first batches of the benchmark
    for i in range(2):
        batch = synth.uniform_keys(K, seed + 40, offset=i * K)
        S, added = orc.insert(S, batch)
        assert c.insert_batch(to_dev(batch)) == added
    check(c, S, orc)

    # range sums: short ranges (~1.5e3 keys) and long ones (~1.5e6 keys, thousands
    # of interior leaves), plus the full range
    for width, n in ((1 << 24, 20000), (1 << 34, 200)):
        lo, hi = synth.range_queries_width(n, seed + 60 + width.bit_length(), width)
        gs, gn = c.range_map(lo, hi)
        es, en = orc.range_map(S, lo, hi)
        assert np.array_equal(gn, en) and np.array_equal(gs, es)
    # the range benchmark's query shape: Zipf(1.2) lengths 1..1e6 as exact key counts
    lens = synth.zipf_lengths(100000, seed + 62, alpha=1.2, lmax=10 ** 6)
    lo, hi = synth.range_queries_by_count(S, lens, seed + 63)
    gs, gn = c.range_map(lo, hi)
    es, en = orc.range_map(S, lo, hi)
    assert np.array_equal(gn, np.minimum(lens, len(S)).astype(np.uint64))
    assert np.array_equal(gn, en) and np.array_equal(gs, es)
    fs, fn = c.range_map(np.array([0], np.uint64), np.array([(1 << 64) - 1], np.uint64))
    es, en = orc.range_map(S, np.array([0], np.uint64), np.array([(1 << 64) - 1], np.uint64))
    assert int(fn[0]) == len(S) and int(fs[0]) == int(es[0])

    # membership: sampled present keys and fresh draws (mostly absent)
    q = np.concatenate([S[synth.sample_indices(len(S), 50000, seed + 70)], synth.uniform_keys(50000, seed + 71)])
    assert np.array_equal(c.contains(q), orc.contains(S, q))

    # a delete batch of 1e7 present keys
    dels = S[synth.sample_indices(len(S), K, seed + 80)]
    S, removed = orc.delete(S, dels)
    assert removed == K
    assert c.delete_batch(to_dev(dels)) == removed
    check(c, S, orc)
