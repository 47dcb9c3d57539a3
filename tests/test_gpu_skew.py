"""Skewed workloads and the growing factor (Section "Evaluation on
microbenchmarks": batches of Zipf-distributed 34-bit keys with skew 0.99 into a
set of uniform 40-bit keys; appendix "Growing factor sensitivity"), and long
insert slices into leaves above 1 KiB.  Every batch is checked against the
oracle and the structure checker."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_05055_amd as p
    p.lib()
    return p


def check(c, expect, orc):
    b, u, h = c.export()
    L, S = c.geometry()
    code, msg = orc.check_image(b, u, h, S, expect)
    assert code == 0, msg
    assert c.size() == len(expect)


@pytest.mark.parametrize("S", [64, 1024])
def test_zipf_insert_delete(cp, orc, S):
    """Zipf(0.99) batches over 34-bit keys: many repeats inside a batch, and the
    distinct keys crowd the low end of the key space, so a few leaves take long
    slices and windows there are redistributed."""
    seed = synth.SEED_BASE + 501
    base = synth.uniform_keys(200000, seed, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=S)
    check(c, expect, orc)
    off = 0
    for step, (kind, k) in enumerate([("ins", 50000), ("ins", 2000), ("del", 20000), ("ins", 100000),
                                      ("del", 3000), ("ins", 4096), ("del", 60000)]):
        batch = synth.zipf_keys(k, seed + 1, offset=off)
        off += k
        if kind == "ins":
            expect, added = orc.insert(expect, batch)
            assert c.insert_batch(batch) == added
        else:
            expect, removed = orc.delete(expect, batch)
            assert c.delete_batch(batch) == removed
        check(c, expect, orc)
    lo = synth.zipf_keys(2000, seed + 2)
    hi = lo + synth.uniform_keys(2000, seed + 3, bits=20)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(n, en)


@pytest.mark.parametrize("grow", [1.1, 1.5, 2.0])
def test_growing_factors(cp, orc, grow):
    """The set grows several times and then shrinks with growing factor 1.1, 1.5
    and 2.0 (the range the paper sweeps); the layout stays within every bound."""
    cfg = cp.default_config()
    cfg.leaf_bytes = 256
    cfg.grow = grow
    cfg.build_density = 0.0  # default: up_root / grow
    seed = synth.SEED_BASE + 601
    base = synth.uniform_keys(40000, seed, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, config=cfg)
    check(c, expect, orc)
    L0 = c.geometry()[0]
    for b in range(5):
        batch = synth.uniform_keys(30000, seed + 10 + b, bits=40)
        expect, added = orc.insert(expect, batch)
        assert c.insert_batch(batch) == added
        check(c, expect, orc)
    L1 = c.geometry()[0]
    assert L1 > 2 * L0
    for b in range(4):
        dels = expect[synth.sample_indices(len(expect), len(expect) // 2, seed + 20 + b)]
        expect, removed = orc.delete(expect, dels)
        assert c.delete_batch(dels) == removed
        check(c, expect, orc)
    assert c.geometry()[0] < L1


@pytest.mark.parametrize("S", [2048, 4096])
def test_long_slices_in_large_leaves(cp, orc, S):
    """Leaves above 1 KiB take the lane merge, and an insert slice of more than
    4096 keys goes to the heavy merge through the staging buffer: a dense run of
    keys between two present keys, then a second run into the leaf it filled."""
    seed = synth.SEED_BASE + 701
    base = synth.uniform_keys(100000, seed, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=S)
    check(c, expect, orc)
    i = len(expect) // 3
    x0 = int(expect[i]) + 1
    gap = (int(expect[i + 1]) - x0) // 20000
    assert gap >= 1
    run1 = np.uint64(x0) + np.arange(6000, dtype=np.uint64) * np.uint64(gap)
    expect, added = orc.insert(expect, run1)
    assert c.insert_batch(run1) == added == 6000
    check(c, expect, orc)
    run2 = run1[:-1] + np.uint64(max(1, gap // 2))      # interleaved with run1: the same leaves
    run2 = np.concatenate([run2, synth.uniform_keys(2000, seed + 1, bits=40)])
    expect, added = orc.insert(expect, run2)
    assert c.insert_batch(run2) == added
    check(c, expect, orc)
    lo = run1[::100]
    hi = lo + np.uint64(50 * gap)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(n, en)
