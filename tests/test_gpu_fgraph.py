"""F-Graph on the GPU CPMA against the CPU oracle: BFS levels bit-exact,
FP32 PageRank within 1e-5 relative of the FP64 oracle."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cp():
    import torch
    assert torch.cuda.is_available()
    import paper_2305_05055_amd as p
    p.lib()
    return p


def graph(scale, samples, seed):
    s, d = synth.rmat_edges(samples, seed, scale=scale)
    return synth.edge_keys(s, d)


def check_graph(c, keys_sorted, nv, orc, src=0, pagerank=True, symmetric=True):
    want = orc.bfs(keys_sorted, nv, src)
    assert np.array_equal(c.bfs(nv, src), want)                    # top-down levels only
    if symmetric:
        assert np.array_equal(c.bfs(nv, src, symmetric=True), want)  # bottom-up where cheaper
    if not pagerank:
        return
    p32 = c.pagerank(nv, iters=10).astype(np.float64)
    p64 = orc.pagerank(keys_sorted, nv, iters=10)
    rel = np.abs(p32 - p64) / p64
    assert rel.max() <= 1e-5, rel.max()


@pytest.mark.parametrize("S", [128, 1024])
def test_bfs_pagerank_small_rmat(cp, orc, S):
    scale = 12
    keys = graph(scale, 30000, 101)
    ks = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=S)
    check_graph(c, ks, 1 << scale, orc)
    check_graph(c, ks, 1 << scale, orc, src=17)


def test_edge_batches_then_algorithms(cp, orc):
    scale = 14
    keys = graph(scale, 100000, 202)
    ks = orc.build_set(keys)
    c = cp.CPMA(keys)
    for b in range(3):
        batch = graph(scale, 20000, 300 + b)
        ks, added = orc.insert(ks, batch)
        assert c.insert_batch(batch) == added
    check_graph(c, ks, 1 << scale, orc)
    fwd = ks[::5]
    rev = ((fwd & np.uint64(0xffffffff)) << np.uint64(32)) | (fwd >> np.uint64(32))
    dels = np.concatenate([fwd, rev])                    # keep the edge set symmetric
    ks, removed = orc.delete(ks, dels)
    assert c.delete_batch(dels) == removed
    check_graph(c, ks, 1 << scale, orc)


def test_disconnected_and_isolated_vertices(cp, orc):
    # two components plus isolated vertices; ids near the top of the range
    nv = 1000
    pairs = [(i, i + 1) for i in range(10)] + [(900, 950), (950, 999)]
    ks = np.array(sorted({(a << 32) | b for a, b in pairs} | {(b << 32) | a for a, b in pairs}),
                  dtype=np.uint64)
    c = cp.CPMA(ks, leaf_bytes=64)
    check_graph(c, ks, nv, orc)
    check_graph(c, ks, nv, orc, src=950)


def test_bfs_directed_edges(cp, orc):
    """BFS follows u -> v on an asymmetric edge set too."""
    nv = 4096
    s, d = synth.rmat_edges(20000, 505, scale=12)
    ks = orc.build_set(synth.edge_keys(s, d, symmetric=False))
    c = cp.CPMA(ks, leaf_bytes=256)
    check_graph(c, ks, nv, orc, pagerank=False, symmetric=False)
    check_graph(c, ks, nv, orc, src=1, pagerank=False, symmetric=False)


def test_rmat_scale20(cp, orc):
    """A larger R-MAT graph drawn on the GPU (same values as the numpy generator)."""
    import torch
    scale = 20
    s, d = synth.rmat_edges_torch(1 << 23, 404, scale=scale, device="cuda")
    dk = synth.edge_keys_torch(s, d)
    c = cp.CPMA(dk)
    ks = orc.build_set(dk.cpu().numpy().view(np.uint64))
    assert c.size() == len(ks)
    check_graph(c, ks, 1 << scale, orc)


def test_rmat_scale24_benchmarked_size(cp, orc):
    """The F-Graph benchmark's graph itself (scale 24, 2^27 samples, ~2.7e8
    symmetric edge keys, drawn on the GPU by the same generator): BFS levels
    from vertex 0 bit-exact in both directions, 10 FP32 PageRank iterations
    within 1e-5 relative of the FP64 oracle."""
    import torch
    scale = 24
    nv = 1 << scale
    s, d = synth.rmat_edges_torch(1 << 27, synth.SEED_BASE + 2 + 60, scale=scale, device="cuda")
    dk = synth.edge_keys_torch(s, d)
    del s, d
    c = cp.CPMA(dk)
    ks = orc.build_set(dk.cpu().numpy().view(np.uint64))
    del dk
    torch.cuda.empty_cache()
    assert c.size() == len(ks)
    check_graph(c, ks, nv, orc)


# ---- vertex offsets, connected components, single-source betweenness --------------
def check_more(c, ks, nv, orc, sources=(0,)):
    assert np.array_equal(c.offsets(nv), orc.offsets(ks, nv))
    assert np.array_equal(c.cc(nv), orc.cc(ks, nv))
    for src in sources:
        sg, dl = c.bc(nv, src)
        osg, odl = orc.bc(ks, nv, src)
        small = osg < 2.0 ** 50                       # path counts exact while well inside FP64
        assert np.array_equal(sg[small], osg[small])
        assert np.allclose(sg[~small], osg[~small], rtol=1e-12, atol=0)
        err = np.abs(dl - odl) / np.maximum(1.0, np.abs(odl))
        assert err.max() <= 1e-9, (src, err.max())


@pytest.mark.parametrize("S", [128, 1024])
def test_offsets_cc_bc_small_rmat(cp, orc, S):
    scale = 12
    keys = graph(scale, 30000, 111)
    ks = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=S)
    check_more(c, ks, 1 << scale, orc, sources=(0, 17, (1 << scale) - 1))


def test_cc_many_components_and_isolated(cp, orc):
    """Several disjoint R-MAT graphs on separate id ranges, plus isolated ids and
    edges whose ids lie beyond nv (ignored)."""
    parts = []
    for i in range(5):
        s, d = synth.rmat_edges(3000, 500 + i, scale=10)
        parts.append(synth.edge_keys(s + np.uint64(2048 * i), d + np.uint64(2048 * i)))
    nv = 5 * 2048 + 100
    beyond = synth.edge_keys(np.array([5, nv + 3], np.uint64), np.array([nv + 7, 9], np.uint64))
    keys = np.concatenate(parts + [beyond])
    ks = orc.build_set(keys)
    c = cp.CPMA(keys, leaf_bytes=256)
    inside = ks[((ks >> np.uint64(32)) < nv) & ((ks & np.uint64(0xffffffff)) < nv)]
    assert np.array_equal(c.cc(nv), orc.cc(inside, nv))
    assert np.array_equal(c.offsets(nv), orc.offsets(inside, nv))
    lab = c.cc(nv, device=True).cpu().numpy().view(np.uint32)
    assert np.array_equal(lab, orc.cc(inside, nv))


def test_erdos_renyi_graph(cp, orc):
    nv = 1 << 15
    s, d = synth.er_edges(200000, 701, nv)
    keys = synth.edge_keys(s, d)
    ks = orc.build_set(keys)
    c = cp.CPMA(keys)
    check_more(c, ks, nv, orc, sources=(0, 12345))
    check_graph(c, ks, nv, orc)


def test_offsets_cc_bc_after_edge_batches(cp, orc):
    scale = 16
    keys = graph(scale, 400000, 811)
    ks = orc.build_set(keys)
    c = cp.CPMA(keys)
    for b in range(2):
        batch = graph(scale, 60000, 820 + b)
        ks, added = orc.insert(ks, batch)
        assert c.insert_batch(batch) == added
    fwd = ks[::7]
    rev = ((fwd & np.uint64(0xffffffff)) << np.uint64(32)) | (fwd >> np.uint64(32))
    ks, removed = orc.delete(ks, np.concatenate([fwd, rev]))
    assert c.delete_batch(np.concatenate([fwd, rev])) == removed
    check_more(c, ks, 1 << scale, orc, sources=(0, 3))
    sg, dl = c.bc(1 << scale, 0, device=True)
    osg, odl = orc.bc(ks, 1 << scale, 0)
    err = np.abs(dl.cpu().numpy() - odl) / np.maximum(1.0, np.abs(odl))
    assert err.max() <= 1e-9
