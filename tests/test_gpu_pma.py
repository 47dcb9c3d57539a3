"""The uncompressed variant (the plain PMA the paper measures compression
against, Section "Packed Memory Array"; compared in Section "Evaluation on
microbenchmarks"): the same batch algorithm on leaves of raw 8-byte keys.
GPU results against the oracle, bit-exact, with the uncompressed checker run
on the exported layout after every batch."""
import ctypes

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
    code, msg = orc.check_image_pma(b, u, h, S, expect, params or orc.DEFAULT_PARAMS)
    assert code == 0, msg
    assert c.size() == len(expect)
    assert c.bytes() == L * (S + 12)


def ranges_agree(c, expect, orc, seed, bits):
    lo = synth.uniform_keys(700, seed, bits=bits)
    hi = lo + synth.uniform_keys(700, seed + 1, bits=max(4, bits - 6))
    lo = np.concatenate([lo, np.array([0, 5, 0], np.uint64)])
    hi = np.concatenate([hi, np.array([M64, 5, 1], np.uint64)])  # everything, empty, [0, 1)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(n, en) and np.array_equal(s, es)
    q = np.concatenate([expect[::97], synth.uniform_keys(500, seed + 2, bits=bits)])
    assert np.array_equal(c.contains(q), orc.contains(expect, q))


@pytest.mark.parametrize("S", [64, 256, 1024])
@pytest.mark.parametrize("n", [0, 1, 9, 1000, 30000])
def test_build(cp, orc, S, n):
    keys = synth.uniform_keys(n, 3100 + n, bits=40)
    if n > 4:
        keys[: n // 4] = keys[n // 4: 2 * (n // 4)]
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=S, uncompressed=True)
    check(c, expect, orc)
    if n:
        ranges_agree(c, expect, orc, 3200 + n, 40)
    c.close()


@pytest.mark.parametrize("S", [64, 512, 4096])
@pytest.mark.parametrize("seed", [1, 2])
def test_insert_delete_sequence(cp, orc, S, seed):
    """Batches from 1 to 20000 keys (the small one-launch preparation below
    4096 keys, the sorted pipeline above it), with growth and shrinking."""
    base = synth.uniform_keys(5000, 3300 + seed, bits=26)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=S, uncompressed=True)
    check(c, expect, orc)
    for step, k in enumerate([1, 7, 300, 20000, 4096, 9000, 3, 12000, 640, 18000]):
        if step % 3 == 2:
            m = min(k, len(expect))
            present = expect[synth.sample_indices(len(expect), m - m // 4, seed * 50 + step)]
            batch = np.concatenate([present, synth.uniform_keys(m // 4, seed * 60 + step, bits=26)])
            new, removed = orc.delete(expect, batch)
            assert c.delete_batch(batch) == removed
        else:
            batch = synth.uniform_keys(k, seed * 70 + step, bits=26)
            r = min(k // 4, len(expect))
            if r:
                batch[:r] = expect[synth.sample_indices(len(expect), r, seed * 80 + step)]
            new, added = orc.insert(expect, batch)
            assert c.insert_batch(batch) == added
        expect = new
        check(c, expect, orc)
    ranges_agree(c, expect, orc, 3400 + seed, 26)
    # delete everything, then refill
    assert c.delete_batch(expect) == len(expect)
    check(c, np.zeros(0, np.uint64), orc)
    refill = synth.uniform_keys(7000, 3500 + seed, bits=26)
    expect, added = orc.insert(np.zeros(0, np.uint64), refill)
    assert c.insert_batch(refill) == added
    check(c, expect, orc)
    c.close()


def test_skewed_batches_redistribute_windows(cp, orc):
    """Batches packed into a narrow key range overfill a few leaves: windows
    are redistributed (and slices far above 64 keys merge into one leaf)."""
    base = synth.uniform_keys(60000, 3600, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=256, uncompressed=True)
    L0 = c.geometry()[0]
    for i in range(6):
        x0 = np.uint64(int(synth.uniform_keys(1, 3610 + i, bits=39)[0]))
        batch = x0 + synth.uniform_keys(2500, 3620 + i, bits=20)
        expect, added = orc.insert(expect, batch)
        assert c.insert_batch(batch) == added
        check(c, expect, orc)
    assert c.geometry()[0] >= L0
    ranges_agree(c, expect, orc, 3630, 40)
    c.close()


@pytest.mark.parametrize("frac", [0.1, 1e9])
def test_rebuild_and_counted_path(cp, orc, frac):
    cfg = cp.default_config()
    cfg.leaf_bytes = 512
    cfg.rebuild_frac = frac
    cfg.uncompressed = 1
    base = synth.uniform_keys(200000, 3700, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, config=cfg)
    for i, k in enumerate([20000, 200000]):
        batch = synth.uniform_keys(k, 3710 + i, bits=40)
        expect, added = orc.insert(expect, batch)
        assert c.insert_batch(batch) == added
        check(c, expect, orc)
        dels = expect[synth.sample_indices(len(expect), k, 3720 + i)]
        expect, removed = orc.delete(expect, dels)
        assert c.delete_batch(dels) == removed
        check(c, expect, orc)
    c.close()


def test_device_batches_noalloc_and_trim(cp, orc):
    import torch
    base = synth.uniform_keys(100000, 3800, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(torch.from_numpy(base.view(np.int64)).cuda(), uncompressed=True)
    batch = synth.uniform_keys(50000, 3801, bits=40)
    expect, added = orc.insert(expect, batch)
    assert c.insert_batch(torch.from_numpy(batch.view(np.int64)).cuda()) == added
    c.trim()
    check(c, expect, orc)
    lo = synth.uniform_keys(3000, 3802, bits=40)
    hi = lo + synth.uniform_keys(3000, 3803, bits=32)
    s, n = c.range_map_noalloc(torch.from_numpy(lo.view(np.int64)).cuda(),
                               torch.from_numpy(hi.view(np.int64)).cuda())
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(n.cpu().numpy().view(np.uint64), en)
    assert np.array_equal(s.cpu().numpy().view(np.uint64), es)
    c.close()


def test_calls_without_uncompressed_support_refuse(cp, orc):
    c = cp.CPMA(synth.uniform_keys(1000, 3900, bits=40), uncompressed=True)
    L = cp.lib()
    lv = np.zeros(16, np.uint32)
    assert L.cpma_fgraph_bfs(c.handle, 16, 0, 1, 0, ctypes.c_void_p(lv.ctypes.data), None) == 1  # CPMA_ERR_INVALID
    with pytest.raises(cp.CpmaError):
        c.apply_updates([(cp.REQ_INSERT, synth.uniform_keys(10, 3901, bits=40))])
    base = cp.default_config()
    base.uncompressed = 1
    with pytest.raises(cp.CpmaError):
        cp.autotune(synth.uniform_keys(100000, 3902, bits=40), base=base)
    # the set is unchanged by the refused calls
    check(c, orc.build_set(synth.uniform_keys(1000, 3900, bits=40)), orc)
    c.close()


def test_bad_flag_value_is_rejected(cp):
    cfg = cp.default_config()
    cfg.uncompressed = 2
    with pytest.raises(cp.CpmaError):
        cp.CPMA(synth.uniform_keys(10, 3950, bits=40), config=cfg)
