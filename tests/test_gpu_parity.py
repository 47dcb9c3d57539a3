"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by
element, with the structure checker run on the exported layout after every batch.

Integer results are bit-exact: set contents, n_added / n_removed, range sums
(mod 2^64) and counts, membership.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def cp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_05055_amd as p
    p.lib()
    return p


def check(c, expect, orc, params=None):
    b, u, h = c.export()
    L, S = c.geometry()
    code, msg = orc.check_image(b, u, h, S, expect, params or orc.DEFAULT_PARAMS)
    assert code == 0, msg
    assert c.size() == len(expect)
    assert c.bytes() == L * (S + 12)


def full_range(c, S_oracle):
    s, n = c.range_map(np.array([0], np.uint64), np.array([M64], np.uint64))
    return int(s[0]), int(n[0])


@pytest.mark.parametrize("S", [64, 256, 1024])
@pytest.mark.parametrize("n", [0, 1, 2, 17, 1000, 20000])
def test_build(cp, orc, S, n):
    keys = synth.uniform_keys(n, 1000 + n, bits=40)
    if n > 4:
        keys[: n // 4] = keys[n // 4: 2 * (n // 4)]  # repeated keys in the input
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=S)
    check(c, expect, orc)
    s, cnt = full_range(c, expect)
    assert cnt == len(expect) and s == int(expect.sum(dtype=np.uint64))


@pytest.mark.parametrize("S", [64, 128, 1024])
@pytest.mark.parametrize("seed", [1, 2])
def test_insert_delete_sequence(cp, orc, S, seed):
    base = synth.uniform_keys(3000, seed, bits=24)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=S)
    check(c, expect, orc)
    for step in range(10):
        k = [1, 7, 100, 900, 2500, 50, 4000, 3, 1200, 640][step]
        if step % 3 == 2:
            # delete: half present keys, half random (mostly absent)
            present = expect[synth.sample_indices(len(expect), min(k // 2, len(expect)), seed * 100 + step)]
            batch = np.concatenate([present, synth.uniform_keys(k - len(present), seed * 77 + step, bits=24)])
            new, removed = orc.delete(expect, batch)
            got = c.delete_batch(batch)
            assert got == removed
        else:
            batch = synth.uniform_keys(k, seed * 1000 + step, bits=24)
            if len(expect) and k > 4:
                batch[: k // 4] = expect[synth.sample_indices(len(expect), k // 4, step)]
            new, added = orc.insert(expect, batch)
            got = c.insert_batch(batch)
            assert got == added
        expect = new
        check(c, expect, orc)
    lo = synth.uniform_keys(500, seed + 5, bits=24)
    hi = lo + synth.uniform_keys(500, seed + 6, bits=16)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(n, en)


@pytest.mark.parametrize("S", [64, 1024])
def test_range_map_edges(cp, orc, S):
    keys = np.concatenate([np.array([0, 1, 2, M64 - 1, M64 - 2, 1 << 63], np.uint64),
                           synth.uniform_keys(5000, 9, bits=64)])
    keys = keys[keys != np.uint64(M64)]
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=S)
    check(c, expect, orc)
    rnd_lo = synth.uniform_keys(2000, 10, bits=64)
    rnd_hi = rnd_lo + synth.uniform_keys(2000, 11, bits=58)
    lo = np.concatenate([np.array([0, 0, 5, 5, M64 - 1, 0, 1 << 63, 3], np.uint64), expect[:50], rnd_lo])
    hi = np.concatenate([np.array([M64, 1, 5, 4, M64, M64 - 1, M64, 2], np.uint64),
                         expect[:50] + np.uint64(1), rnd_hi])
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(n, en)
    assert np.array_equal(s, es)


@pytest.mark.parametrize("S", [64, 1024])
def test_contains(cp, orc, S):
    keys = synth.uniform_keys(30000, 21, bits=32)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=S)
    q = np.concatenate([expect[::7], synth.uniform_keys(3000, 22, bits=32),
                        np.array([0, M64 - 1], np.uint64)])
    assert np.array_equal(c.contains(q), orc.contains(expect, q))


def test_plain_cpma_config(cp, orc):
    """1e6 uniform 40-bit keys, 10 inserts of 1e4, a delete of 1e4 present keys,
    1e4 range sums over [lo, lo + 2^24): everything bit-exact."""
    seed = synth.SEED_BASE + 1
    keys = synth.unique_uniform_keys(10 ** 6, seed)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys)
    check(c, expect, orc)
    for b in range(10):
        batch = synth.uniform_keys(10 ** 4, seed + 100 + b)
        expect, added = orc.insert(expect, batch)
        assert c.insert_batch(batch) == added
    idx = synth.sample_indices(len(expect), 10 ** 4, seed + 200)
    dbatch = expect[idx]
    expect, removed = orc.delete(expect, dbatch)
    assert removed == 10 ** 4
    assert c.delete_batch(dbatch) == removed
    check(c, expect, orc)
    lo, hi = synth.range_queries_width(10 ** 4, seed + 300, 1 << 24)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(n, en) and np.array_equal(s, es)


def test_heavy_slice_sequential_batch(cp, orc):
    """A batch whose keys all land in one leaf (more than the in-LDS slice)."""
    base = synth.uniform_keys(20000, 31, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base)
    x0 = int(expect[5000]) + 1
    batch = np.arange(x0, x0 + 6000, dtype=np.uint64)
    expect, added = orc.insert(expect, batch)
    assert c.insert_batch(batch) == added
    check(c, expect, orc)
    batch2 = np.arange(0, 3000, dtype=np.uint64) * np.uint64(3)  # below every key
    expect, added = orc.insert(expect, batch2)
    assert c.insert_batch(batch2, sorted=True) == added
    check(c, expect, orc)


def skewed_batch(expect, sizes, seed):
    """Clusters of consecutive keys, each starting just above a present key (so
    each cluster lands in one leaf), with every fourth cluster key replaced by a
    present key of the set."""
    rng = np.random.default_rng(seed)
    parts = []
    starts = rng.choice(len(expect) - 1, size=len(sizes), replace=False)
    for st, nb in zip(starts, sizes):
        x0 = int(expect[st]) + 1
        gap = max(1, (int(expect[st + 1]) - x0) // (2 * nb + 1))
        cl = np.uint64(x0) + np.arange(nb, dtype=np.uint64) * np.uint64(gap)
        pres = expect[st: st + (nb + 3) // 4]
        cl[::4] = pres[: len(cl[::4])]
        parts.append(cl)
    batch = np.concatenate(parts)
    rng.shuffle(batch)
    return batch


@pytest.mark.parametrize("S", [64, 1024])
@pytest.mark.parametrize("sizes", [[65, 100, 300, 700, 1024], [1025, 1700, 2500, 65, 4096]])
def test_skewed_insert_slices(cp, orc, sizes, S):
    """Few long insert slices (65 to 4096 keys): each goes to the one-wave heavy
    merge, through LDS up to 1024 keys and through the staging buffer above
    (with 64-byte leaves every such leaf overflows into the arena)."""
    base = synth.uniform_keys(200000, 71, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=S)
    for seed in (1, 2):
        batch = skewed_batch(expect, sizes, seed)
        expect, added = orc.insert(expect, batch)
        assert c.insert_batch(batch) == added
        check(c, expect, orc)
    # a small batch (the one-launch path) with the same shape
    batch = skewed_batch(expect, [70, 1200, 300], 3)
    assert len(batch) <= 4096
    expect, added = orc.insert(expect, batch)
    assert c.insert_batch(batch) == added
    check(c, expect, orc)


def test_many_spilled_slices(cp, orc):
    """A batch as large as the set: every leaf gets a slice of more than 64 keys,
    and all of them (thousands) go to the one-wave heavy merge, through LDS or
    the staging buffer."""
    base = synth.uniform_keys(1_000_000, 73, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base)
    L, _ = c.geometry()
    assert L > 2048
    batch = np.concatenate([synth.uniform_keys(900_000, 74, bits=40),
                            skewed_batch(expect, [400, 900, 2000], 5)])
    expect, added = orc.insert(expect, batch)
    assert c.insert_batch(batch) == added
    check(c, expect, orc)


def test_first_batches_locate_per_key(cp, orc):
    """The first updates of a freshly built set are batches above the one-launch
    size but below the leaf count, so the batch keys are located one by one
    (and every per-batch buffer of that branch is sized by the batch itself)."""
    base = synth.uniform_keys(2_000_000, 43, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=64)
    assert c.geometry()[0] > 20000
    batch = synth.uniform_keys(6000, 44, bits=40)
    expect, added = orc.insert(expect, batch)
    assert c.insert_batch(batch) == added
    check(c, expect, orc)
    dels = np.concatenate([expect[::400], synth.uniform_keys(1000, 45, bits=40)])
    expect, removed = orc.delete(expect, dels)
    assert c.delete_batch(dels) == removed
    check(c, expect, orc)


@pytest.mark.parametrize("p", [63, 64 * 4 * 4096 - 1])
def test_single_descent_detected(cp, orc, p):
    """A batch sorted except for one adjacent pair, placed where the sortedness
    check takes the right neighbour from another wave (and, for the second
    position, from the next grid-stride round): it must be sorted."""
    keys = orc.build_set(synth.uniform_keys(1_100_000, 47, bits=40))
    keys[p], keys[p + 1] = keys[p + 1], keys[p]
    base = orc.build_set(synth.uniform_keys(50_000, 48, bits=40))
    c = cp.CPMA(base)
    expect, added = orc.insert(base, keys)
    assert c.insert_batch(keys) == added
    check(c, expect, orc)


def test_phase_statistics_select(cp, orc):
    """Phase timing: a selected phase alone accumulates launches, time and bytes;
    the others stay zero; all phases when enabled; a mask bit past the last
    phase is rejected."""
    import ctypes
    base = synth.uniform_keys(200_000, 49, bits=40)
    c = cp.CPMA(base)
    c.stats_select(["merge"])
    c.insert_batch(synth.uniform_keys(100_000, 50, bits=40))
    st = c.stats()
    assert st["merge"][0] == 1 and st["merge"][1] > 0 and st["merge"][2] > 0
    assert all(v == (0, 0.0, 0) for name, v in st.items() if name != "merge")
    c.stats_enable(True)
    c.insert_batch(synth.uniform_keys(100_000, 51, bits=40))
    st = c.stats()
    for name in ("sort", "locate", "merge", "count"):
        assert st[name][0] >= 1 and st[name][1] > 0, name
    c.stats_enable(False)
    assert cp.lib().cpma_stats_select(c._h, ctypes.c_uint32(1 << 8)) == 1


@pytest.mark.parametrize("k", [2, 3, 63, 64, 65, 127, 128, 129, 511, 1000, 1024, 1025, 4096])
def test_small_batch_sorting(cp, orc, k):
    """Batches of the one-launch path, across the sort's shapes (in-wave and LDS
    stages, one key per thread or several): random order with repeats, and
    reversed order."""
    base = synth.uniform_keys(20_000, 70 + k, bits=30)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=256)
    batch = synth.uniform_keys(k, 71 + k, bits=30)
    batch[: k // 3] = batch[k // 3: 2 * (k // 3)]  # repeats
    expect, added = orc.insert(expect, batch)
    assert c.insert_batch(batch) == added
    check(c, expect, orc)
    present = expect[:: max(1, len(expect) // (k - k // 2))][: k - k // 2]
    rev = orc.build_set(np.concatenate([synth.uniform_keys(k // 2, 72 + k, bits=30), present]))[::-1].copy()
    expect, removed = orc.delete(expect, rev)
    assert c.delete_batch(rev) == removed
    check(c, expect, orc)


def test_many_small_batches(cp, orc):
    """Many small batches in a row (the one-launch preparation): dense runs
    overflow leaves and windows (redistribution, growth), scattered keys touch
    one leaf each, and deletes of contiguous runs empty regions (lower bounds):
    the structure is checked after every batch."""
    base = synth.uniform_keys(30_000, 81, bits=32)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=256)
    for step in range(45):
        kind = step % 3
        if kind == 0:      # a dense run of new keys inside one key range
            x0 = int(synth.uniform_keys(1, 900 + step, bits=32)[0])
            batch = np.arange(x0, x0 + 3 * 60, 3, dtype=np.uint64)
        elif kind == 1:    # scattered keys
            batch = synth.uniform_keys(20, 900 + step, bits=32)
        else:              # deletes of a contiguous run of present keys
            i0 = int(synth.uniform_keys(1, 900 + step, bits=20)[0]) % max(1, len(expect) - 200)
            batch = expect[i0:i0 + 150].copy()
        if kind == 2:
            expect, n = orc.delete(expect, batch)
            assert c.delete_batch(batch) == n
        else:
            expect, n = orc.insert(expect, batch)
            assert c.insert_batch(batch) == n
        check(c, expect, orc)


@pytest.mark.parametrize("S,n0", [(64, 5000), (1024, 50000), (1024, 3)])
def test_small_batch_path_counts(cp, orc, S, n0):
    """Small batches count only the paths of the touched leaves while every node
    was within bounds before them; a batch that pushes a path node out of bounds,
    a resize, a large batch and deletes that shrink the set all hand over to the
    full count.  The density bounds of every node are checked after each batch."""
    rng = np.random.default_rng(S + n0)
    expect = orc.build_set(synth.uniform_keys(n0, 91, bits=36))
    c = cp.CPMA(expect, leaf_bytes=S)
    for step in range(40):
        r = step % 8
        if r == 5:      # a large batch (the full pipeline and the full count)
            batch = synth.uniform_keys(6000, 950 + step, bits=36)
        elif r == 6 and len(expect) > 100:  # deletes of a run, then of scattered keys
            i0 = int(rng.integers(0, len(expect) - 50))
            batch = np.concatenate([expect[i0:i0 + 50], rng.choice(expect, size=min(300, len(expect) // 3))])
        elif r in (2, 3):  # a dense run: overfills a leaf and its window
            x0 = int(synth.uniform_keys(1, 950 + step, bits=36)[0])
            batch = np.arange(x0, x0 + 2 * 200, 2, dtype=np.uint64)
        else:           # scattered keys, 1 to 4096 of them
            batch = synth.uniform_keys(int(rng.choice([1, 7, 100, 1000, 4096])), 950 + step, bits=36)
        if r == 6:
            expect, n = orc.delete(expect, batch)
            assert c.delete_batch(batch) == n
        else:
            expect, n = orc.insert(expect, batch)
            assert c.insert_batch(batch) == n
        check(c, expect, orc)


def test_delete_all_then_reinsert(cp, orc):
    keys = synth.uniform_keys(5000, 41, bits=40)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=128)
    assert c.delete_batch(expect[::-1].copy()) == len(expect)
    check(c, np.empty(0, np.uint64), orc)
    assert c.range_map(np.array([0], np.uint64), np.array([M64], np.uint64))[1][0] == 0
    assert c.insert_batch(keys) == len(expect)
    check(c, expect, orc)


def test_repeats_present_keys_and_empty_batches(cp, orc):
    keys = synth.uniform_keys(4000, 51, bits=20)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=256)
    assert c.insert_batch(np.empty(0, np.uint64)) == 0
    assert c.delete_batch(np.empty(0, np.uint64)) == 0
    assert c.insert_batch(np.repeat(expect[:100], 3)) == 0       # all present, repeated
    absent = np.setdiff1d(synth.uniform_keys(500, 52, bits=20), expect)
    assert c.delete_batch(absent) == 0
    check(c, expect, orc)


def test_reserved_key_rejected_and_set_unchanged(cp, orc):
    keys = synth.uniform_keys(1000, 61, bits=40)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys)
    bad = np.array([5, M64, 7], dtype=np.uint64)
    with pytest.raises(cp.CpmaError) as e:
        c.insert_batch(bad)
    assert e.value.code == 4
    with pytest.raises(cp.CpmaError):
        c.delete_batch(bad)
    check(c, expect, orc)
    with pytest.raises(cp.CpmaError):
        cp.CPMA(bad)


def test_large_batches_sorted_or_reserved(cp, orc):
    """Batches large enough that their first radix pass is queued before the
    validation result is known: one holding the reserved key (rejected, set
    unchanged, the same batch then accepted without it), and an already sorted
    one (the queued pass is unused)."""
    base = synth.uniform_keys(300_000, 63, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base)
    bad = synth.uniform_keys(200_000, 64, bits=40)
    bad[123_456] = M64
    with pytest.raises(cp.CpmaError) as e:
        c.insert_batch(bad)
    assert e.value.code == 4
    with pytest.raises(cp.CpmaError):
        c.delete_batch(bad)
    check(c, expect, orc)
    good = np.delete(bad, 123_456)
    expect, added = orc.insert(expect, good)
    assert c.insert_batch(good) == added
    check(c, expect, orc)
    srt = orc.build_set(synth.uniform_keys(150_000, 65, bits=40))
    expect, added = orc.insert(expect, srt)
    assert c.insert_batch(srt) == added  # sorted input, sorted flag not given
    check(c, expect, orc)
    expect, removed = orc.delete(expect, srt[::2])
    assert c.delete_batch(srt[::2]) == removed
    check(c, expect, orc)


def test_growth_and_shrink_tiny_leaves(cp, orc):
    """64-byte leaves: many resizes up, then deletes shrink the array again."""
    c = cp.CPMA(np.empty(0, np.uint64), leaf_bytes=64)
    expect = np.empty(0, np.uint64)
    for b in range(12):
        batch = synth.uniform_keys(300 * (b + 1), 70 + b, bits=40)
        expect, added = orc.insert(expect, batch)
        assert c.insert_batch(batch) == added
        check(c, expect, orc)
    L_big = c.geometry()[0]
    for b in range(6):
        idx = synth.sample_indices(len(expect), len(expect) // 2, 90 + b)
        dbatch = expect[idx]
        expect, removed = orc.delete(expect, dbatch)
        assert c.delete_batch(dbatch) == removed
        check(c, expect, orc)
    assert c.geometry()[0] < L_big


def test_device_tensors(cp, orc):
    import torch
    keys = synth.uniform_keys(50000, 81, bits=40)
    expect = orc.build_set(keys)
    dev = torch.from_numpy(keys.view(np.int64)).cuda()
    c = cp.CPMA(dev)
    check(c, expect, orc)
    batch = synth.uniform_keys(20000, 82, bits=40)
    expect, added = orc.insert(expect, batch)
    assert c.insert_batch(torch.from_numpy(batch.view(np.int64)).cuda()) == added
    lo, hi = synth.range_queries_width(3000, 83, 1 << 30)
    s, n = c.range_map(torch.from_numpy(lo.view(np.int64)).cuda(), torch.from_numpy(hi.view(np.int64)).cuda())
    torch.cuda.synchronize()
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s.cpu().numpy().view(np.uint64), es)
    assert np.array_equal(n.cpu().numpy().view(np.uint64), en)
    q = torch.from_numpy(np.concatenate([expect[:1000], batch[:1000] + np.uint64(1)]).view(np.int64)).cuda()
    got = c.contains(q).cpu().numpy()
    assert np.array_equal(got, orc.contains(expect, q.cpu().numpy().view(np.uint64)))
    check(c, expect, orc)


def test_allocator_hooks(cp, orc):
    """cpma_config.alloc / free: every device buffer of the handle comes from the
    hooks and goes back at destroy; an allocator that runs out makes the build
    fail with CPMA_ERR_NOMEM and returns what it had taken."""
    import ctypes
    import torch
    ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
    FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
    live, budget = {}, [None]

    def _alloc(n, ctx):
        if budget[0] is not None and sum(live.values()) + n > budget[0]:
            return None
        p = torch.cuda.caching_allocator_alloc(n)
        live[p] = n
        return p

    def _free(p, ctx):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    a_cb, f_cb = ALLOC(_alloc), FREE(_free)
    cfg = cp.default_config()
    cfg.leaf_bytes = 256
    cfg.alloc = ctypes.cast(a_cb, ctypes.c_void_p).value
    cfg.free = ctypes.cast(f_cb, ctypes.c_void_p).value
    keys = synth.uniform_keys(100000, 71, bits=40)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, config=cfg)
    assert live
    for b in range(3):  # grows the array several times
        batch = synth.uniform_keys(100000, 72 + b, bits=40)
        expect, added = orc.insert(expect, batch)
        assert c.insert_batch(batch) == added
    dels = expect[synth.sample_indices(len(expect), 50000, 75)]
    expect, removed = orc.delete(expect, dels)
    assert c.delete_batch(dels) == removed
    check(c, expect, orc)
    lo, hi = synth.range_queries_width(1000, 76, 1 << 30)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(n, en) and np.array_equal(s, es)
    c.close()
    assert not live
    budget[0] = 1 << 20  # far below what 1e5 keys need
    with pytest.raises(cp.CpmaError) as e:
        cp.CPMA(keys, config=cfg)
    assert e.value.code == 2
    assert not live


@pytest.mark.parametrize("bounds", [None, (0.99, 0.90, 0.10, 0.30)])
def test_dense_leaves(cp, orc, bounds):
    """Leaves of 1-byte codes at their density bounds (up to about a thousand
    keys in a 1 KiB leaf, the most the wave merge's key array holds): inserts
    concentrated in one key range (large batches, then small ones) fill its
    leaves, then deletes hit them, each batch checked against the oracle."""
    params = bounds or orc.DEFAULT_PARAMS
    base = np.arange(0, 400000, 2, dtype=np.uint64)  # gap 2: every code one byte
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=1024, bounds=bounds)
    check(c, expect, orc, params)
    odd = np.arange(1, 80000, 2, dtype=np.uint64)  # the dense range: [0, 80000)
    rng = np.random.default_rng(5)
    rng.shuffle(odd)
    # a leaf of 1-byte codes holds used - 7 keys; batches must meet leaves of
    # more than 768 keys (more than 896 with the looser bounds)
    dense = 903 if bounds else 775
    seen = 0
    pos = 0
    for k in [8000, 8000, 8000, 6000, 4000, 2000, 1000, 1000, 500, 64, 7]:
        batch = odd[pos:pos + k]
        pos += k
        new, added = orc.insert(expect, batch)
        assert c.insert_batch(batch) == added
        expect = new
        check(c, expect, orc, params)
        _, u, _ = c.export()
        seen = max(seen, int(u.max()))
    assert seen > dense
    dense_keys = expect[expect < np.uint64(80000)]
    for k in [5000, 3000, 700, 60, 5]:
        batch = dense_keys[synth.sample_indices(len(dense_keys), k, 900 + k)]
        new, removed = orc.delete(expect, batch)
        assert c.delete_batch(batch) == removed
        expect = new
        dense_keys = expect[expect < np.uint64(80000)]
        check(c, expect, orc, params)
    lo = np.arange(0, 400000, 9973, dtype=np.uint64)
    hi = lo + np.uint64(50000)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(n, en)
