"""The full rebuild of large batches (Section "Parallel Batch Updates in a
PMA": a batch of at least about n / 10 keys rebuilds the whole structure):
batches at k = n / 10 and k = n, inserts and deletes, with the rebuild and
with the counted batch path, against the oracle and the structure checker."""
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
    return L


@pytest.mark.parametrize("S", [256, 1024])
@pytest.mark.parametrize("frac", [0.1, 1e9])   # rebuild at n / 10, or never
def test_rebuild_at_tenth_and_whole(cp, orc, S, frac):
    cfg = cp.default_config()
    cfg.leaf_bytes = S
    cfg.rebuild_frac = frac
    seed = synth.SEED_BASE + 1101
    base = synth.uniform_keys(300000, seed, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, config=cfg)
    check(c, expect, orc)
    n = len(expect)
    steps = [("ins", n // 10), ("ins", n), ("del", n // 10), ("ins", n // 10 + 7), ("del", n)]
    rebuilt = 0
    for i, (kind, k) in enumerate(steps):
        size_before = len(expect)
        if kind == "ins":
            batch = synth.uniform_keys(k, seed + 10 + i, bits=40)
            batch[: k // 5] = expect[synth.sample_indices(len(expect), k // 5, seed + 20 + i)]  # some present
            expect, added = orc.insert(expect, batch)
            assert c.insert_batch(batch) == added
        else:
            m = min(k, len(expect))
            batch = np.concatenate([expect[synth.sample_indices(len(expect), m, seed + 30 + i)],
                                    synth.uniform_keys(k // 10, seed + 40 + i, bits=40)])
            expect, removed = orc.delete(expect, batch)
            assert c.delete_batch(batch) == removed
        L = check(c, expect, orc)
        if len(batch) >= frac * size_before and len(expect):
            # a rebuild leaves the layout at about the build density
            rebuilt += 1
            b, u, h = c.export()
            dens = float(u.astype(np.float64).sum()) / (L * S)
            assert abs(dens - cfg.build_density) < 0.05, (i, dens)
    assert rebuilt == (3 if frac < 1 else 0)
    lo = synth.uniform_keys(3000, seed + 50, bits=40)
    hi = lo + synth.uniform_keys(3000, seed + 51, bits=30)
    s, cnt = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(cnt, en)


def test_rebuild_deletes_everything_then_refills(cp, orc):
    cfg = cp.default_config()
    cfg.leaf_bytes = 256
    base = synth.uniform_keys(50000, 1201, bits=40)
    expect = orc.build_set(base)
    c = cp.CPMA(base, config=cfg)
    assert c.delete_batch(expect) == len(expect)
    check(c, np.empty(0, np.uint64), orc)
    assert c.size() == 0 and c.geometry()[0] == 1
    expect, added = orc.insert(np.empty(0, np.uint64), base[:20000])
    assert c.insert_batch(base[:20000]) == added
    check(c, expect, orc)
    # a fused update call above the threshold takes the rebuild as well
    ins = synth.uniform_keys(30000, 1202, bits=40)
    dels = expect[::2]
    res = c.apply_updates([(cp.REQ_DELETE, dels), (cp.REQ_INSERT, ins)])
    e1, r1 = orc.delete(expect, dels)
    e2, a2 = orc.insert(e1, ins)
    assert list(res) == [r1, a2]
    check(c, e2, orc)
