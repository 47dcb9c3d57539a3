"""The key-value CPMA (every key carries an 8-byte value; the extension the
paper names for weighted graphs, Section "Evaluation on graph workloads").
GPU results against the oracle's key-value set, bit-exact, with the key-value
checker run on the exported layout after every batch."""
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


def check(c, K, V, orc):
    b, u, h = c.export()
    L, S = c.geometry()
    code, msg = orc.check_image_kv(b, u, c.code_bytes(), h, S, K, V)
    assert code == 0, msg
    assert c.size() == len(K)
    assert c.bytes() == L * (S + 16)


def queries_agree(c, K, V, orc, seed, bits):
    lo = synth.uniform_keys(600, seed, bits=bits)
    hi = lo + synth.uniform_keys(600, seed + 1, bits=max(4, bits - 5))
    lo = np.concatenate([lo, np.array([0, 9, 0], np.uint64)])
    hi = np.concatenate([hi, np.array([M64, 9, 1], np.uint64)])
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(K, lo, hi)
    assert np.array_equal(n, en) and np.array_equal(s, es)
    vs, vn = c.range_map_values(lo, hi)
    evs, evn = orc.kv_range_values(K, V, lo, hi)
    assert np.array_equal(vn, evn) and np.array_equal(vs, evs)
    q = np.concatenate([K[::53], synth.uniform_keys(400, seed + 2, bits=bits)])
    val, found = c.get(q)
    eval_, efound = orc.kv_get(K, V, q)
    assert np.array_equal(found, efound) and np.array_equal(val, eval_)
    assert np.array_equal(c.contains(q), efound)


def values_for(keys, seed):
    return synth.uniform_keys(len(keys), seed, bits=64)


@pytest.mark.parametrize("S", [64, 256, 1024])
@pytest.mark.parametrize("n", [0, 1, 9, 1000, 30000])
def test_build(cp, orc, S, n):
    keys = synth.uniform_keys(n, 4100 + n, bits=40)
    if n > 4:
        keys[: n // 4] = keys[n // 4: 2 * (n // 4)]  # repeats: the first occurrence's value counts
    vals = values_for(keys, 4150 + n)
    K, V = orc.kv_build(keys, vals)
    c = cp.CPMA(keys, leaf_bytes=S, values=vals)
    check(c, K, V, orc)
    if n:
        queries_agree(c, K, V, orc, 4200 + n, 40)
    c.close()


@pytest.mark.parametrize("S", [128, 1024, 4096])
@pytest.mark.parametrize("seed", [1, 2])
def test_upsert_insert_delete_sequence(cp, orc, S, seed):
    """Upserts (new and present keys, repeats), key-only inserts and deletes of
    1 to 20000 keys, through growth and shrinking."""
    base = synth.uniform_keys(5000, 4300 + seed, bits=26)
    K, V = orc.kv_build(base, values_for(base, 4310 + seed))
    c = cp.CPMA(base, leaf_bytes=S, values=values_for(base, 4310 + seed))
    check(c, K, V, orc)
    for step, k in enumerate([1, 9, 300, 20000, 5000, 8000, 3, 12000, 700, 18000]):
        kind = step % 4
        keys = synth.uniform_keys(k, seed * 90 + step, bits=26)
        r = min(k // 3, len(K))
        if r:
            keys[:r] = K[synth.sample_indices(len(K), r, seed * 91 + step)]
        if kind == 3:
            K, V, removed = orc.kv_delete(K, V, keys)
            assert c.delete_batch(keys) == removed
        elif kind == 2:
            # key-only insert: new keys get 0, present keys keep their value
            zeros = np.zeros(len(keys), np.uint64)
            bk, bv = orc.kv_build(keys, zeros)
            new = ~np.isin(bk, K)
            K2, V2, added = orc.kv_insert(K, V, bk[new], bv[new])
            assert c.insert_batch(keys) == added
            K, V = K2, V2
        else:
            vals = values_for(keys, seed * 92 + step)
            K, V, added = orc.kv_insert(K, V, keys, vals)
            assert c.insert_kv(keys, vals) == added
        check(c, K, V, orc)
    queries_agree(c, K, V, orc, 4400 + seed, 26)
    K2, V2, removed = orc.kv_delete(K, V, K)
    assert c.delete_batch(K) == removed
    check(c, K2, V2, orc)
    refill = synth.uniform_keys(7000, 4450 + seed, bits=26)
    rv = values_for(refill, 4460 + seed)
    K, V, added = orc.kv_insert(K2, V2, refill, rv)
    assert c.insert_kv(refill, rv) == added
    check(c, K, V, orc)
    c.close()


def test_skewed_upserts_overflow_leaves_and_windows(cp, orc):
    """Batches packed into one narrow key range: merged leaves overflow into the
    arena (more than a thousand keys into one leaf) and windows redistribute."""
    base = synth.uniform_keys(60000, 4500, bits=40)
    K, V = orc.kv_build(base, values_for(base, 4501))
    c = cp.CPMA(base, leaf_bytes=512, values=values_for(base, 4501))
    for i in range(5):
        x0 = np.uint64(int(synth.uniform_keys(1, 4510 + i, bits=39)[0]))
        keys = x0 + synth.uniform_keys(3000, 4520 + i, bits=18)
        vals = values_for(keys, 4530 + i)
        K, V, added = orc.kv_insert(K, V, keys, vals)
        assert c.insert_kv(keys, vals) == added
        check(c, K, V, orc)
    queries_agree(c, K, V, orc, 4540, 40)
    c.close()


@pytest.mark.parametrize("frac", [0.1, 1e9])
def test_rebuild_and_counted_path(cp, orc, frac):
    cfg = cp.default_config()
    cfg.leaf_bytes = 1024
    cfg.rebuild_frac = frac
    base = synth.uniform_keys(150000, 4600, bits=40)
    K, V = orc.kv_build(base, values_for(base, 4601))
    c = cp.CPMA(base, config=cfg, values=values_for(base, 4601))
    for i, k in enumerate([20000, 150000]):
        keys = synth.uniform_keys(k, 4610 + i, bits=40)
        keys[: k // 2] = K[synth.sample_indices(len(K), k // 2, 4615 + i)]
        vals = values_for(keys, 4620 + i)
        K, V, added = orc.kv_insert(K, V, keys, vals)
        assert c.insert_kv(keys, vals) == added
        check(c, K, V, orc)
        dels = K[synth.sample_indices(len(K), k, 4630 + i)]
        K, V, removed = orc.kv_delete(K, V, dels)
        assert c.delete_batch(dels) == removed
        check(c, K, V, orc)
    c.close()


def test_weighted_graph_degrees_and_bfs(cp, orc):
    """A weighted F-Graph: edge keys u << 32 | v carrying weights.  The weighted
    degree of every vertex is range_map_values over [u << 32, (u + 1) << 32);
    BFS runs on the same set as on an unweighted one."""
    scale = 12
    nv = 1 << scale
    src, dst = synth.rmat_edges(nv * 8, 4700, scale=scale)
    ekeys = synth.edge_keys(src, dst)
    w = synth.uniform_keys(len(ekeys), 4701, bits=20)
    K, V = orc.kv_build(ekeys, w)
    c = cp.CPMA(ekeys, values=w)
    check(c, K, V, orc)
    lo = (np.arange(nv, dtype=np.uint64) << np.uint64(32))
    hi = lo + (np.uint64(1) << np.uint64(32))
    ws, deg = c.range_map_values(lo, hi)
    ews, edeg = orc.kv_range_values(K, V, lo, hi)
    assert np.array_equal(deg, edeg) and np.array_equal(ws, ews)
    assert np.array_equal(c.bfs(nv, 0, symmetric=True), orc.bfs(K, nv, 0))
    # reweight a sample of edges, remove others, and check again
    pick = K[synth.sample_indices(len(K), 5000, 4702)]
    nw = synth.uniform_keys(len(pick), 4703, bits=20)
    K, V, added = orc.kv_insert(K, V, pick, nw)
    assert added == 0 and c.insert_kv(pick, nw) == 0
    gone = K[synth.sample_indices(len(K), 3000, 4704)]
    K, V, removed = orc.kv_delete(K, V, gone)
    assert c.delete_batch(gone) == removed
    check(c, K, V, orc)
    ws, deg = c.range_map_values(lo, hi)
    ews, edeg = orc.kv_range_values(K, V, lo, hi)
    assert np.array_equal(deg, edeg) and np.array_equal(ws, ews)
    c.close()


def test_device_buffers_noalloc_and_trim(cp, orc):
    import torch
    keys = synth.uniform_keys(80000, 4800, bits=40)
    vals = values_for(keys, 4801)
    K, V = orc.kv_build(keys, vals)
    tk = torch.from_numpy(keys.view(np.int64)).cuda()
    tv = torch.from_numpy(vals.view(np.int64)).cuda()
    c = cp.CPMA(tk, values=tv)
    more = synth.uniform_keys(40000, 4802, bits=40)
    mv = values_for(more, 4803)
    K, V, added = orc.kv_insert(K, V, more, mv)
    assert c.insert_kv(torch.from_numpy(more.view(np.int64)).cuda(),
                       torch.from_numpy(mv.view(np.int64)).cuda()) == added
    c.trim()
    check(c, K, V, orc)
    q = torch.from_numpy(K[::7].view(np.int64)).cuda()
    val, found = c.get(q)
    assert found.cpu().numpy().all()
    assert np.array_equal(val.cpu().numpy().view(np.uint64), V[::7])
    lo = synth.uniform_keys(2000, 4804, bits=40)
    hi = lo + synth.uniform_keys(2000, 4805, bits=30)
    s, n = c.range_map_noalloc(torch.from_numpy(lo.view(np.int64)).cuda(), torch.from_numpy(hi.view(np.int64)).cuda())
    es, en = orc.range_map(K, lo, hi)
    assert np.array_equal(s.cpu().numpy().view(np.uint64), es) and np.array_equal(n.cpu().numpy().view(np.uint64), en)
    c.close()


def test_calls_without_value_support_refuse(cp, orc):
    keys = synth.uniform_keys(1000, 4900, bits=40)
    c = cp.CPMA(keys, values=values_for(keys, 4901))
    with pytest.raises(cp.CpmaError):
        c.apply_updates([(cp.REQ_INSERT, synth.uniform_keys(10, 4902, bits=40))])
    base = cp.default_config()
    base.values = 1
    with pytest.raises(cp.CpmaError):
        cp.autotune(synth.uniform_keys(100000, 4903, bits=40), base=base)
    plain = cp.CPMA(keys)
    with pytest.raises(cp.CpmaError):
        plain.get(keys[:5])
    with pytest.raises(cp.CpmaError):
        plain.range_map_values(keys[:5], keys[:5] + np.uint64(1))
    with pytest.raises(cp.CpmaError):
        plain.insert_kv(keys[:5], keys[:5])
    cfg = cp.default_config()
    cfg.uncompressed = 1
    with pytest.raises(cp.CpmaError):
        cp.CPMA(keys, config=cfg, values=keys)
    K, V = orc.kv_build(keys, values_for(keys, 4901))
    check(c, K, V, orc)
    c.close()
    plain.close()
