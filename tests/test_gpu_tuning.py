"""GPU: the autotuner, leaf sizes up to 4 KB, the range-scan chunk, and a
range_map batch captured in a HIP graph and replayed -- every result against the
CPU oracle (bit-exact), every layout through the structure checker."""
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
    code, msg = orc.check_image(b, u, h, S, expect, orc.DEFAULT_PARAMS)
    assert code == 0, msg


def test_autotune_report_and_tuned_set(cp, orc):
    keys = synth.uniform_keys(1_500_000, 71, bits=40)
    cfg, rep = cp.autotune(keys, batch=100_000, range_keys=200, queries=20_000, sample_keys=1 << 18)
    assert rep["best_leaf_bytes"] in (256, 512, 1024, 2048, 4096)
    assert rep["best_chunk"] in (1, 2, 4, 8, 16, 32)
    assert cfg.leaf_bytes == rep["best_leaf_bytes"] and cfg.range_chunk == rep["best_chunk"]
    assert 1 << 16 <= rep["sample_n"] <= 1 << 20
    for S, t in rep["leaf_bytes"].items():
        assert t["insert_ms"] > 0 and t["range_ms"] > 0
    # the rebuild cut-over: batches of this relative size rebuild iff that was faster
    assert rep["rebuild_ms"] > 0 and rep["batch_path_ms"] > 0
    r = 100_000 / 1_500_000
    assert cfg.rebuild_frac == rep["best_rebuild_frac"]
    if rep["rebuild_ms"] < rep["batch_path_ms"]:
        assert cfg.rebuild_frac <= r * (1 + 1e-9)
    else:
        assert cfg.rebuild_frac >= 2 * r * (1 - 1e-9)
    # the tuned configuration gives a valid set with oracle-exact results
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, config=cfg)
    check(c, expect, orc)
    batch = synth.uniform_keys(100_000, 72, bits=40)
    expect, added = orc.insert(expect, batch)
    assert c.insert_batch(batch) == added
    check(c, expect, orc)
    lo = synth.uniform_keys(5000, 73, bits=40)
    hi = lo + np.uint64(1 << 28)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(n, en)


def test_autotune_rejects_bad_input(cp):
    with pytest.raises(cp.CpmaError):
        cp.autotune(np.array([1, 2, (1 << 64) - 1], np.uint64))
    with pytest.raises(cp.CpmaError):
        cp.autotune(np.array([], np.uint64))


@pytest.mark.parametrize("S", [2048, 4096])
def test_large_leaves_sequence(cp, orc, S):
    base = synth.uniform_keys(200_000, 80 + S, bits=36)
    expect = orc.build_set(base)
    c = cp.CPMA(base, leaf_bytes=S)
    check(c, expect, orc)
    for step, k in enumerate([10, 5000, 120_000, 70, 30_000]):
        if step % 2:
            batch = np.concatenate([expect[synth.sample_indices(len(expect), k // 2, step)],
                                    synth.uniform_keys(k - k // 2, 90 + step, bits=36)])
            expect, removed = orc.delete(expect, batch)
            assert c.delete_batch(batch) == removed
        else:
            batch = synth.uniform_keys(k, 95 + step, bits=36)
            expect, added = orc.insert(expect, batch)
            assert c.insert_batch(batch) == added
        check(c, expect, orc)
    lo = synth.uniform_keys(3000, 99, bits=36)
    hi = lo + synth.uniform_keys(3000, 98, bits=30)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(n, en)


@pytest.mark.parametrize("chunk", [1, 64])
def test_range_chunk(cp, orc, chunk):
    keys = synth.uniform_keys(400_000, 110, bits=40)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, range_chunk=chunk)
    lens = synth.zipf_lengths(4000, 111, alpha=1.2, lmax=100_000)
    lo, hi = synth.range_queries_by_count(expect, lens, 112)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(expect, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(n, en)
    assert np.array_equal(n, np.minimum(lens, len(expect)).astype(np.uint64))


def test_bad_range_chunk_rejected(cp):
    with pytest.raises(cp.CpmaError):
        cp.CPMA(np.arange(10, dtype=np.uint64), range_chunk=3)


def test_range_map_graph_capture(cp, orc):
    """A range_map batch on device buffers, captured once and replayed with new
    query contents written into the same buffers between replays."""
    import torch
    keys = synth.uniform_keys(300_000, 120, bits=40)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys)
    q = 20_000
    lo_t = torch.zeros(q, dtype=torch.int64, device="cuda")
    hi_t = torch.zeros(q, dtype=torch.int64, device="cuda")

    def fill(seed):
        lo = synth.uniform_keys(q, seed, bits=40)
        hi = lo + synth.uniform_keys(q, seed + 1, bits=32)
        lo_t.copy_(torch.from_numpy(lo.view(np.int64)))
        hi_t.copy_(torch.from_numpy(hi.view(np.int64)))
        return lo, hi

    fill(130)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        c.range_map(lo_t, hi_t)   # warm-up: sizes the scratch buffers
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s_t, n_t = c.range_map(lo_t, hi_t)
    for rep in range(4):
        lo, hi = fill(140 + 2 * rep)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        es, en = orc.range_map(expect, lo, hi)
        assert np.array_equal(s_t.cpu().numpy().view(np.uint64), es)
        assert np.array_equal(n_t.cpu().numpy().view(np.uint64), en)
        # eager call in between, same buffers
        s2, n2 = c.range_map(lo_t, hi_t)
        assert np.array_equal(s2.cpu().numpy().view(np.uint64), es)
