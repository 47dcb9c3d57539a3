"""Pins for the CPU oracle: each check ties it to something other than itself.

* set algebra vs. Python's own set type on random small inputs (brute force);
* range sums vs. closed forms (arithmetic series, full range = total, empty
  ranges) and vs. a predicate scan;
* the byte codec vs. published LEB128 byte patterns (tests/golden);
* the structure checker vs. a hand-built image (tests/golden) and planted
  mistakes in it;
* PageRank / BFS vs. graph special cases with known answers.
"""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
M64 = (1 << 64) - 1


# --------------------------------------------------------------------------- sets
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n,k", [(0, 0), (0, 7), (1, 1), (50, 20), (700, 300), (2000, 2000)])
def test_set_ops_match_python_sets(orc, seed, n, k):
    rng = np.random.default_rng(seed)
    space = max(8, 3 * (n + k))
    base = rng.integers(0, space, size=n, dtype=np.uint64)
    batch = rng.integers(0, space, size=k, dtype=np.uint64)
    S = orc.build_set(base)
    assert S.tolist() == sorted(set(base.tolist()))
    ins, added = orc.insert(S, batch)
    ref = set(S.tolist()) | set(batch.tolist())
    assert ins.tolist() == sorted(ref)
    assert added == len(set(batch.tolist()) - set(S.tolist()))
    dele, removed = orc.delete(ins, batch[: k // 2])
    ref2 = ref - set(batch[: k // 2].tolist())
    assert dele.tolist() == sorted(ref2)
    assert removed == len(set(batch[: k // 2].tolist()) & ref)
    q = rng.integers(0, space, size=64, dtype=np.uint64)
    assert orc.contains(ins, q).tolist() == [int(x in ref) for x in q.tolist()]


def test_insert_then_delete_restores_set(orc):
    S = orc.build_set(synth.uniform_keys(5000, 11))
    B = synth.uniform_keys(3000, 12)
    ins, added = orc.insert(S, B)
    assert len(ins) == len(S) + added
    fresh = np.setdiff1d(B, S)
    back, removed = orc.delete(ins, fresh)
    assert removed == added
    assert np.array_equal(back, S)


# ------------------------------------------------------------------------ ranges
def test_range_closed_form_arithmetic_series(orc):
    S = np.arange(1000, 3001, dtype=np.uint64)  # keys a..b
    lo = np.array([1000, 0, 1500, 1500, 2000, 5000, 3001], dtype=np.uint64)
    hi = np.array([3001, 10 ** 6, 1501, 1500, 1000, 6000, 4000], dtype=np.uint64)
    s, c = orc.range_map(S, lo, hi)
    for i in range(len(lo)):
        a = max(1000, int(lo[i]))
        b = min(3000, int(hi[i]) - 1)
        if int(lo[i]) >= int(hi[i]) or a > b:
            assert (s[i], c[i]) == (0, 0)
        else:
            assert int(c[i]) == b - a + 1
            assert int(s[i]) == ((a + b) * (b - a + 1) // 2) % (1 << 64)


def test_range_full_equals_total_and_wraps(orc):
    top = M64 - 5
    S = orc.build_set(np.array([top - 3 * i for i in range(50)], dtype=np.uint64))
    s, c = orc.range_map(S, np.array([0], dtype=np.uint64), np.array([M64], dtype=np.uint64))
    assert int(c[0]) == 50
    assert int(s[0]) == sum(int(x) for x in S) % (1 << 64)


@pytest.mark.parametrize("seed", range(4))
def test_range_matches_predicate_scan(orc, seed):
    S = orc.build_set(synth.uniform_keys(800, 100 + seed, bits=16))
    lo = synth.uniform_keys(300, 200 + seed, bits=16)
    w = synth.uniform_keys(300, 300 + seed, bits=12)
    hi = lo + w
    hi[:10] = lo[:10]                      # empty
    hi[10:20] = lo[10:20] - np.uint64(1)   # lo > hi
    s1, c1 = orc.range_map(S, lo, hi)
    s2, c2 = orc.range_map(S, lo, hi, brute=True)
    assert np.array_equal(s1, s2) and np.array_equal(c1, c2)
    s3, c3 = orc.range_map(S, lo, hi, threads=7)   # uneven blocks
    assert np.array_equal(s3, s2) and np.array_equal(c3, c2)
    assert (c1[:20] == 0).all() and (s1[:20] == 0).all()


# ------------------------------------------------------------------------- codec
def _golden_leb():
    rows = []
    with open(os.path.join(GOLDEN, "leb128_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows.append((int(parts[0]), bytes(int(x, 16) for x in parts[1:])))
    return rows


def test_codec_published_patterns(orc):
    rows = _golden_leb()
    assert len(rows) >= 7
    for v, b in rows:
        assert orc.varint_encode(v) == b
        assert orc.varint_decode(b) == (v, len(b))


def test_codec_length_boundaries_and_roundtrip(orc):
    vals = [1, M64, M64 - 1]
    for j in range(1, 10):
        vals += [(1 << (7 * j)) - 1, 1 << (7 * j)]
    for v in vals:
        b = orc.varint_encode(v)
        assert len(b) == -(-v.bit_length() // 7)          # ceil(bitlen / 7)
        assert all(x & 0x80 for x in b[:-1]) and not (b[-1] & 0x80)
        assert b[-1] != 0                                  # terminator never 0x00
        assert orc.varint_decode(b) == (v, len(b))
        assert orc.varint_decode(b[:-1])[1] == -1          # truncated code rejected
    assert orc.varint_encode(M64) == bytes([0xFF] * 9 + [0x01])


# ------------------------------------------------------------------------ bounds
def test_bounds_match_hand_computed_table(orc):
    """Every interior bound, not only the ends, against the table worked out by
    hand in tests/golden/density_bounds_table.txt (H = 3, 5, 19)."""
    rows = 0
    with open(os.path.join(GOLDEN, "density_bounds_table.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            H, which, *vals = line.split()
            H = int(H)
            assert len(vals) == H + 1
            w = 0 if which == "up" else 1
            assert [orc.bound_q(w, h, H) for h in range(H + 1)] == [int(v) for v in vals]
            rows += 1
    assert rows == 6


def test_bounds_interpolate_between_leaf_and_root(orc):
    for H in (0, 1, 5, 19):
        ups = [orc.bound_q(0, h, H) for h in range(H + 1)]
        los = [orc.bound_q(1, h, H) for h in range(H + 1)]
        assert ups[0] == round(0.9 * 65536) and los[0] == round(0.1 * 65536)
        if H > 0:
            assert ups[-1] == round(0.7 * 65536) and los[-1] == round(0.3 * 65536)
        assert all(a >= b for a, b in zip(ups, ups[1:]))
        assert all(a <= b for a, b in zip(los, los[1:]))
    assert [orc.tree_height(L) for L in (1, 2, 3, 4, 5, 1024, 1025)] == [0, 1, 2, 2, 3, 10, 11]


# ----------------------------------------------------------------------- checker
def _golden_image(name="leaf_image_s64.txt"):
    S = None
    params = None
    keys = []
    leaves = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, *rest = line.split()
            if tag == "S":
                S = int(rest[0])
            elif tag == "params":
                params = tuple(float(x) for x in rest)
            elif tag == "keys":
                keys = [int(x) for x in rest]
            elif tag == "leaf":
                leaves.append(bytes(int(x, 16) for x in rest))
    L = len(leaves)
    img = np.zeros(L * S, dtype=np.uint8)
    used = np.zeros(L, dtype=np.uint32)
    head = np.zeros(L, dtype=np.uint64)
    for i, lf in enumerate(leaves):
        img[i * S:i * S + len(lf)] = np.frombuffer(lf, dtype=np.uint8)
        used[i] = len(lf)
        head[i] = int.from_bytes(lf[:8], "little")
    return S, params, np.array(keys, dtype=np.uint64), img, used, head


def test_checker_accepts_golden_image(orc):
    S, params, keys, img, used, head = _golden_image()
    code, msg = orc.check_image(img, used, head, S, keys, params)
    assert code == 0, msg
    assert orc.decode_image(img, used, S, 100).tolist() == keys.tolist()


def test_checker_rejects_planted_mistakes(orc):
    S, params, keys, img, used, head = _golden_image()

    def bad(mut):
        i2, u2, h2, k2 = img.copy(), used.copy(), head.copy(), keys.copy()
        mut(i2, u2, h2, k2)
        code, _ = orc.check_image(i2, u2, h2, S, k2, params)
        return code

    assert bad(lambda i, u, h, k: i.__setitem__(9, 0x82)) != 0          # continue bit flipped on
    assert bad(lambda i, u, h, k: i.__setitem__(8, 0x2c)) != 0          # continue bit flipped off
    assert bad(lambda i, u, h, k: i.__setitem__(40, 0x01)) != 0         # garbage past used
    assert bad(lambda i, u, h, k: h.__setitem__(1, 4999)) != 0          # head index stale
    assert bad(lambda i, u, h, k: u.__setitem__(0, 12)) != 0            # used too short
    assert bad(lambda i, u, h, k: k.__setitem__(2, 1302)) != 0          # content differs
    # leaf 1 starting below leaf 0's last key breaks global order
    assert bad(lambda i, u, h, k: (i.__setitem__(slice(64, 72), np.frombuffer(
        (1200).to_bytes(8, "little"), dtype=np.uint8)), h.__setitem__(1, 1200))) != 0
    # density: default bounds (root lower 0.30) reject the 23/128 root
    code, msg = orc.check_image(img, used, head, S, keys)
    assert code != 0 and "lower" in msg
    # a leaf above 0.9 * 64 bytes violates the leaf upper bound
    big = np.zeros(64, dtype=np.uint8)
    big[:8] = np.frombuffer((7).to_bytes(8, "little"), dtype=np.uint8)
    big[8:60] = 1                                                       # 52 deltas of 1
    ks = np.arange(7, 7 + 53, dtype=np.uint64)
    code, msg = orc.check_image(big, np.array([60], np.uint32), np.array([7], np.uint64), 64, ks)
    assert code != 0 and "upper" in msg
    big[8:57] = 1
    big[57:60] = 0
    ks = np.arange(7, 7 + 50, dtype=np.uint64)
    code, msg = orc.check_image(big, np.array([57], np.uint32), np.array([7], np.uint64), 64, ks)
    assert code == 0, msg                                                # 57 <= 57.6


def _edit_leaf(img, used, keys, leaf, S, new_used=None, append=None, step=1):
    """Shrinks leaf `leaf` of a golden image to new_used bytes (cut at a code
    boundary) or appends `append` one-byte deltas of `step`; returns new
    (img, used, keys)."""
    img, used = img.copy(), used.copy()
    ks = keys.tolist()
    base = leaf * S
    first = sum(_leaf_key_count(img, used, j, S) for j in range(leaf))
    cnt = _leaf_key_count(img, used, leaf, S)
    mine = ks[first:first + cnt]
    u = int(used[leaf])
    if new_used is not None:
        assert img[base + new_used - 1] < 0x80 or new_used == 8  # a code ends there
        img[base + new_used:base + u] = 0
        used[leaf] = new_used
        mine = mine[:_leaf_key_count(img, used, leaf, S)]
    if append:
        img[base + u:base + u + append] = step
        mine = mine + [mine[-1] + step * (j + 1) for j in range(append)]
        used[leaf] = u + append
    ks = ks[:first] + mine + ks[first + cnt:]
    return img, used, np.array(ks, dtype=np.uint64)


def _leaf_key_count(img, used, j, S):
    u = int(used[j])
    if u == 0:
        return 0
    codes = img[j * S + 8:j * S + u]
    return 1 + int(np.count_nonzero(codes < 0x80))  # one terminator per code


def test_checker_accepts_multilevel_golden_image(orc):
    """Five leaves, H = 3: windows at h = 1, 2 and the root are close to their
    bounds, with truncated last windows; the hand-worked figures are in the
    fixture's header.  A checker that measured a truncated window against the
    full 2^h * S bytes, or took H = floor(log2 L), would reject this image."""
    S, params, keys, img, used, head = _golden_image("window_image_l5_s64.txt")
    assert len(used) == 5 and used.tolist() == [48, 47, 48, 47, 20]
    assert params == (0.90, 0.70, 0.10, 0.30)
    code, msg = orc.check_image(img, used, head, S, keys)
    assert code == 0, msg
    assert orc.decode_image(img, used, S, 1000).tolist() == keys.tolist()


def test_checker_multilevel_plants_rejected_for_their_reason(orc):
    S, params, keys, img, used, head = _golden_image("window_image_l5_s64.txt")

    def check(i2, u2, k2, h2=None):
        return orc.check_image(i2, u2, head if h2 is None else h2, S, k2)

    # interior window above its bound: leaves 0 and 1 grow to 55 bytes each
    # (within 57.6 at the leaves), [0,2) = 110 > 106.7 at h = 1
    i2, u2, k2 = _edit_leaf(img, used, keys, 0, S, append=7, step=5)
    i2, u2, k2 = _edit_leaf(i2, u2, k2, 1, S, append=8, step=7)
    assert u2.tolist()[:2] == [55, 55]
    code, msg = check(i2, u2, k2)
    assert code == 13 and msg.startswith("upper density bound violated") and "(1, 0)" in msg, msg
    # truncated last window below its lower bound: leaf 4 keeps its head and
    # one code, 9 bytes: 9 / 64 >= 0.10 at the leaf, < 10.7 bytes at h = 1
    i2, u2, k2 = _edit_leaf(img, used, keys, 4, S, new_used=9)
    code, msg = check(i2, u2, k2)
    assert code == 14 and msg.startswith("lower density bound violated") and "(1, 4)" in msg, msg
    # the root alone above its bound: leaf 4 grows to 40 bytes (within 49.1
    # bytes for [4,5) at h = 2), the root holds 230 > 224.0
    i2, u2, k2 = _edit_leaf(img, used, keys, 4, S, append=20, step=1)
    code, msg = check(i2, u2, k2)
    assert code == 13 and "(3, 0)" in msg, msg
    # the root alone below its bound: leaves 0..3 shrink to 16 bytes each
    # ([0,2) = 32 >= 21.3, [0,4) = 64 >= 59.7), the root holds 84 < 96.0
    i2, u2, k2 = img, used, keys
    for j in range(4):
        i2, u2, k2 = _edit_leaf(i2, u2, k2, j, S, new_used=16)
    code, msg = check(i2, u2, k2)
    assert code == 14 and "(3, 0)" in msg, msg
    # an empty leaf in a set of more than one leaf (its head takes the next
    # leaf's head, the empty-leaf convention): rejected as an empty leaf
    i2, u2, k2 = _edit_leaf(img, used, keys, 2, S, new_used=8)
    i2[2 * S:3 * S] = 0
    u2[2] = 0
    k2 = np.array([k for k in k2.tolist() if k != 3000], dtype=np.uint64)
    h2 = head.copy()
    h2[2] = h2[3]
    code, msg = check(i2, u2, k2, h2)
    assert code == 3 and msg.startswith("empty leaf"), msg


# ------------------------------------------------------------------------- graph
def _sym(pairs):
    ks = set()
    for u, v in pairs:
        if u != v:
            ks.add((u << 32) | v)
            ks.add((v << 32) | u)
    return np.array(sorted(ks), dtype=np.uint64)


def test_pagerank_regular_graphs_stay_uniform(orc):
    n = 64
    cycle = _sym([(i, (i + 1) % n) for i in range(n)])
    clique = _sym([(i, j) for i in range(12) for j in range(i + 1, 12)])
    for e, nv in ((cycle, n), (clique, 12)):
        p = orc.pagerank(e, nv, iters=10)
        assert np.allclose(p, 1.0 / nv, rtol=1e-14, atol=0)


def test_pagerank_star_one_step_closed_form(orc):
    nv, d = 9, 0.85
    e = _sym([(0, i) for i in range(1, nv)])
    p = orc.pagerank(e, nv, iters=1, damping=d)
    center = (1 - d) / nv + d * (nv - 1) * (1.0 / nv)
    leaf = (1 - d) / nv + d * (1.0 / nv) / (nv - 1)
    assert abs(p[0] - center) < 1e-15 and np.allclose(p[1:], leaf, rtol=1e-14)


def test_pagerank_mass_identity(orc):
    nv, d = 300, 0.85
    src, dst = synth.rmat_edges(2000, 5, scale=8)
    e = np.unique(synth.edge_keys(src, dst))
    e = e[(e >> np.uint64(32)) < nv]
    e = e[(e & np.uint64(0xffffffff)) < nv]
    p0 = orc.pagerank(e, nv, iters=3, damping=d)
    p1 = orc.pagerank(e, nv, iters=4, damping=d)
    deg = np.bincount((e >> np.uint64(32)).astype(np.int64), minlength=nv)
    expect = (1 - d) + d * p0[deg > 0].sum()
    assert abs(p1.sum() - expect) < 1e-12


def test_bfs_special_graphs(orc):
    path = _sym([(i, i + 1) for i in range(19)])
    assert orc.bfs(path, 20).tolist() == list(range(20))
    star = _sym([(0, i) for i in range(1, 10)])
    lv = orc.bfs(star, 12)
    assert lv.tolist()[:10] == [0] + [1] * 9 and lv[10] == lv[11] == 0xFFFFFFFF


def test_bfs_matches_python_bfs(orc):
    src, dst = synth.rmat_edges(3000, 9, scale=10)
    e = np.unique(synth.edge_keys(src, dst))
    nv = 1024
    adj = {}
    for x in e.tolist():
        adj.setdefault(x >> 32, []).append(x & 0xffffffff)
    ref = [0xFFFFFFFF] * nv
    ref[0] = 0
    frontier = [0]
    while frontier:
        nxt = []
        for u in frontier:
            for v in adj.get(u, []):
                if ref[v] == 0xFFFFFFFF:
                    ref[v] = ref[u] + 1
                    nxt.append(v)
        frontier = nxt
    assert orc.bfs(e, nv).tolist() == ref


# ------------------------------------------------ vertex offsets, CC, BC (F-Graph)
def test_offsets_star_and_degree_prefix(orc):
    star = _sym([(0, i) for i in range(1, 10)])
    assert orc.offsets(star, 12).tolist() == [0, 9] + list(range(10, 19)) + [18, 18]
    src, dst = synth.rmat_edges(5000, 31, scale=10)
    e = np.unique(synth.edge_keys(src, dst))
    deg = np.bincount((e >> np.uint64(32)).astype(np.int64), minlength=1024)
    assert orc.offsets(e, 1024).tolist() == [0] + np.cumsum(deg).tolist()


def test_cc_known_components_and_union_find(orc):
    pairs = [(i, j) for i in range(3, 8) for j in range(i + 1, 8)]          # clique 3..7
    pairs += [(10, 11), (11, 12), (12, 9)]                                   # path 9..12
    pairs += [(20, 15)]                                                      # edge 15-20
    lab = orc.cc(_sym(pairs), 22)
    want = list(range(22))
    for v in range(3, 8):
        want[v] = 3
    for v in (9, 10, 11, 12):
        want[v] = 9
    want[20] = 15
    assert lab.tolist() == want
    # a random sparse graph against a union-find written here
    src, dst = synth.rmat_edges(3000, 41, scale=11)
    e = np.unique(synth.edge_keys(src, dst))
    nv = 2048
    parent = list(range(nv))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for x in e.tolist():
        a, b = find(x >> 32), find(x & 0xffffffff)
        if a != b:
            parent[max(a, b)] = min(a, b)
    roots = [find(v) for v in range(nv)]
    lo = {}
    for v in range(nv):
        lo.setdefault(roots[v], v)          # smallest id of each set (ids visited in order)
    assert orc.cc(e, nv).tolist() == [lo[roots[v]] for v in range(nv)]


def test_bc_closed_forms(orc):
    n = 12
    sg, dl = orc.bc(_sym([(i, i + 1) for i in range(n - 1)]), n, 0)          # path from an end
    assert sg.tolist() == [1.0] * n and dl.tolist() == [float(n - 1 - v) for v in range(n)]
    sg, dl = orc.bc(_sym([(0, 1), (0, 2), (1, 3), (2, 3)]), 5, 0)          # diamond + isolated 4
    assert sg.tolist() == [1, 1, 1, 2, 0] and dl.tolist() == [3.0, 0.5, 0.5, 0.0, 0.0]
    sg, dl = orc.bc(_sym([(0, i) for i in range(1, 9)]), 9, 0)              # star from its centre
    assert dl.tolist() == [8.0] + [0.0] * 8
    sg, dl = orc.bc(_sym([(0, i) for i in range(1, 9)]), 9, 3)              # star from a leaf
    assert dl[3] == 8.0 and dl[0] == 7.0 and all(dl[v] == 0 for v in range(9) if v not in (0, 3))


def test_bc_brute_force_path_counts(orc):
    """delta_s(v) = sum over t != v of sigma_sv * sigma_vt / sigma_st over the t
    with d(s, v) + d(v, t) = d(s, t): all-pairs distances and path counts by a
    breadth-first search from every vertex, on small random graphs."""
    for seed in (3, 4, 5):
        src, dst = synth.rmat_edges(150, seed, scale=6)
        e = np.unique(synth.edge_keys(src, dst))
        nv = 64
        adj = [[] for _ in range(nv)]
        for x in e.tolist():
            adj[x >> 32].append(x & 0xffffffff)
        D, C = [], []
        for s0 in range(nv):
            d = [-1] * nv
            c = [0] * nv
            d[s0], c[s0] = 0, 1
            fr = [s0]
            while fr:
                nxt = []
                for u in fr:
                    for w in adj[u]:
                        if d[w] < 0:
                            d[w] = d[u] + 1
                            nxt.append(w)
                        if d[w] == d[u] + 1:
                            c[w] += c[u]
                fr = nxt
            D.append(d)
            C.append(c)
        for s0 in (0, 7):
            sg, dl = orc.bc(e, nv, s0)
            for v in range(nv):
                assert sg[v] == C[s0][v]
                want = 0.0
                if D[s0][v] >= 0:
                    for t in range(nv):
                        if t != v and D[s0][t] >= 0 and D[v][t] >= 0 and D[s0][v] + D[v][t] == D[s0][t]:
                            want += C[s0][v] * C[v][t] / C[s0][t]
                assert abs(dl[v] - want) <= 1e-12 * max(1.0, want), (seed, s0, v, dl[v], want)


# ---- the uncompressed variant's checker (the plain PMA) ----------------------------
def _pma_image(leaves, S=64):
    """Hand-built image of the uncompressed layout: each leaf's keys as 8-byte
    little-endian words from its start, zero bytes after them."""
    L = len(leaves)
    img = np.zeros(L * S, dtype=np.uint8)
    used = np.zeros(L, dtype=np.uint32)
    head = np.full(L, np.iinfo(np.uint64).max, dtype=np.uint64)
    for j, ks in enumerate(leaves):
        for t, k in enumerate(ks):
            img[j * S + 8 * t: j * S + 8 * t + 8] = np.frombuffer(int(k).to_bytes(8, "little"), dtype=np.uint8)
        used[j] = 8 * len(ks)
        if ks:
            head[j] = ks[0]
    keys = np.array([k for ks in leaves for k in ks], dtype=np.uint64)
    return img, used, head, keys


# Three leaves of 64 bytes, H = 2, bounds 0.9 / 0.7 (upper, leaf / root) and
# 0.1 / 0.3 (lower), so at h = 1 the bounds are 0.8 and 0.2.  Filled bytes
# 32, 24, 16: leaves 0.5 / 0.375 / 0.25; [0, 2) 56 / 128 = 0.4375; the
# truncated window [2, 3) 16 / 64 = 0.25 (against the full 128 bytes it would
# be 0.125, below 0.2); root 72 / 192 = 0.375.
PMA_GOLDEN = [[10, 20, 30, 40], [50, 60, 70], [80, 90]]


def test_pma_checker_accepts_hand_built_image(orc):
    img, used, head, keys = _pma_image(PMA_GOLDEN)
    code, msg = orc.check_image_pma(img, used, head, 64, keys)
    assert code == 0, msg
    # the same image is no valid delta-coded leaf set (its words are not codes)
    assert orc.check_image(img, used, head, 64, keys)[0] != 0


def test_pma_checker_plants_rejected_for_their_reason(orc):
    S = 64
    # a used count that is not a whole number of keys
    img, used, head, keys = _pma_image(PMA_GOLDEN)
    used[1] = 20
    code, msg = orc.check_image_pma(img, used, head, S, keys)
    assert code == 15, msg
    # keys out of order inside a leaf (the head stays the leaf's first word)
    img, used, head, keys = _pma_image([[10, 30, 20, 40], [50, 60, 70], [80, 90]])
    code, msg = orc.check_image_pma(img, used, head, S, np.sort(keys))
    assert code == 10, msg
    # a head that is not the leaf's first key
    img, used, head, keys = _pma_image(PMA_GOLDEN)
    head[1] = 55
    code, msg = orc.check_image_pma(img, used, head, S, keys)
    assert code == 6, msg
    # a nonzero byte in the free part of a leaf
    img, used, head, keys = _pma_image(PMA_GOLDEN)
    img[2 * S + 20] = 1
    code, msg = orc.check_image_pma(img, used, head, S, keys)
    assert code == 8 and "(2, 20)" in msg, msg
    # a full leaf: 64 / 64 > 0.9 at the leaf level
    img, used, head, keys = _pma_image([[1, 2, 3, 4, 5, 6, 7, 8], [50, 60, 70], [80, 90]])
    code, msg = orc.check_image_pma(img, used, head, S, keys)
    assert code == 13 and "(0, 0)" in msg, msg
    # the truncated last window below 0.2 at h = 1: leaf 2 keeps one key,
    # 8 / 64 = 0.125 (the leaf itself is within 0.1, the root at 64 / 192)
    img, used, head, keys = _pma_image([[10, 20, 30, 40], [50, 60, 70], [80]])
    code, msg = orc.check_image_pma(img, used, head, S, keys)
    assert code == 14 and "(1, 2)" in msg, msg
    # an empty leaf in a set of more than one leaf
    img, used, head, keys = _pma_image([[10, 20, 30, 40], [], [80, 90]])
    code, msg = orc.check_image_pma(img, used, head, S, keys)
    assert code == 3, msg
    # contents that differ from the expected set
    img, used, head, keys = _pma_image(PMA_GOLDEN)
    code, msg = orc.check_image_pma(img, used, head, S, keys + np.uint64(1))
    assert code == 12, msg


# ---- key-value sets: the oracle's upsert semantics and the leaf checker -------------
def _kv_dict_replay(ops):
    """Brute force with a Python dict: ('i', keys, vals) upserts (first
    occurrence of a repeated key in a batch wins), ('d', keys) deletes."""
    d = {}
    counts = []
    for op in ops:
        if op[0] == "i":
            seen = set()
            added = 0
            for k, v in zip(op[1].tolist(), op[2].tolist()):
                if k in seen:
                    continue
                seen.add(k)
                if k not in d:
                    added += 1
                d[k] = v
            counts.append(added)
        else:
            removed = 0
            for k in set(op[1].tolist()):
                if k in d:
                    del d[k]
                    removed += 1
            counts.append(removed)
    return d, counts


def test_kv_oracle_matches_dict_brute_force(orc):
    rng = np.random.default_rng(5)
    K = np.zeros(0, np.uint64)
    V = np.zeros(0, np.uint64)
    ops = []
    got = []
    for step in range(12):
        if step % 3 == 2:
            keys = rng.integers(0, 300, size=40, dtype=np.uint64)
            ops.append(("d", keys))
            K, V, r = orc.kv_delete(K, V, keys)
        else:
            keys = rng.integers(0, 300, size=60, dtype=np.uint64)
            vals = rng.integers(0, 1 << 63, size=60, dtype=np.uint64)
            ops.append(("i", keys, vals))
            K, V, r = orc.kv_insert(K, V, keys, vals)
        got.append(r)
    d, counts = _kv_dict_replay(ops)
    assert got == counts
    assert K.tolist() == sorted(d) and V.tolist() == [d[k] for k in sorted(d)]
    q = np.arange(0, 310, dtype=np.uint64)
    val, found = orc.kv_get(K, V, q)
    assert found.tolist() == [1 if int(x) in d else 0 for x in q]
    assert val.tolist() == [d.get(int(x), 0) for x in q]
    lo = rng.integers(0, 300, size=50, dtype=np.uint64)
    hi = lo + rng.integers(0, 80, size=50, dtype=np.uint64)
    vs, vc = orc.kv_range_values(K, V, lo, hi)
    for a, b, s_, c_ in zip(lo.tolist(), hi.tolist(), vs.tolist(), vc.tolist()):
        inside = [k for k in d if a <= k < b]
        assert c_ == len(inside) and s_ == sum(d[k] for k in inside) % (1 << 64)
    # values equal to the keys: the value sums are the key sums of the set oracle
    vs, vc = orc.kv_range_values(K, K, lo, hi)
    ks, kc = orc.range_map(K, lo, hi)
    assert np.array_equal(vs, ks) and np.array_equal(vc, kc)


def _kv_image(leaves, S=64):
    """Hand-built key-value image: per leaf (keys, values); the head as 8 bytes
    LE, the deltas as LEB128 codes (all below 128 here, one byte each), the
    values as 8-byte LE words at the end of the leaf."""
    L = len(leaves)
    img = np.zeros(L * S, dtype=np.uint8)
    used = np.zeros(L, dtype=np.uint32)
    clen = np.zeros(L, dtype=np.uint32)
    head = np.full(L, np.iinfo(np.uint64).max, dtype=np.uint64)
    for j, (ks, vs) in enumerate(leaves):
        base = j * S
        if not ks:
            continue
        img[base: base + 8] = np.frombuffer(int(ks[0]).to_bytes(8, "little"), dtype=np.uint8)
        p = 8
        for a, b in zip(ks, ks[1:]):
            assert 0 < b - a < 128
            img[base + p] = b - a
            p += 1
        m = len(ks)
        for t, v in enumerate(vs):
            o = base + S - 8 * m + 8 * t
            img[o: o + 8] = np.frombuffer(int(v).to_bytes(8, "little"), dtype=np.uint8)
        clen[j] = p
        used[j] = p + 8 * m
        head[j] = ks[0]
    keys = np.array([k for ks, _ in leaves for k in ks], dtype=np.uint64)
    vals = np.array([v for _, vs in leaves for v in vs], dtype=np.uint64)
    return img, used, clen, head, keys, vals


# Two leaves of 64 bytes, H = 1 (bounds 0.9 / 0.7 upper, 0.1 / 0.3 lower):
# leaf 0 keys 100, 103, 110 (8 + 2 code bytes, 3 values: 34 bytes), leaf 1 keys
# 200, 201 (8 + 1, 2 values: 25 bytes); leaves 0.53 and 0.39, root 59 / 128
# = 0.46.
KV_GOLDEN = [([100, 103, 110], [7, 1 << 40, 9]), ([200, 201], [0, 5])]


def test_kv_checker_accepts_hand_built_image(orc):
    img, used, clen, head, keys, vals = _kv_image(KV_GOLDEN)
    assert used.tolist() == [34, 25] and clen.tolist() == [10, 9]
    code, msg = orc.check_image_kv(img, used, clen, head, 64, keys, vals)
    assert code == 0, msg


def test_kv_checker_plants_rejected_for_their_reason(orc):
    S = 64
    img, used, clen, head, keys, vals = _kv_image(KV_GOLDEN)
    code, msg = orc.check_image_kv(img, used, clen, head, S, keys, vals + np.uint64(1))
    assert code == 18, msg                                    # a wrong value
    u2 = used.copy()
    u2[1] = 26
    code, msg = orc.check_image_kv(img, u2, clen, head, S, keys, vals)
    assert code == 17, msg                                    # used != codes + 8 per key
    c2 = clen.copy()
    c2[0] = 40
    code, msg = orc.check_image_kv(img, used, c2, head, S, keys, vals)
    assert code == 16, msg                                    # codes beyond used
    i2 = img.copy()
    i2[20] = 3                                                # between leaf 0's codes and values
    code, msg = orc.check_image_kv(i2, used, clen, head, S, keys, vals)
    assert code == 8 and "(0, 20)" in msg, msg
    i2 = img.copy()
    i2[9] = 0x80 | 7                                          # a code that runs into the gap
    code, msg = orc.check_image_kv(i2, used, clen, head, S, keys, vals)
    assert code == 5, msg
    # a leaf above its bound: 6 keys (8 + 5 + 48 = 61 > 57.6 bytes)
    img, used, clen, head, keys, vals = _kv_image([([1, 2, 3, 4, 5, 6], [0] * 6), ([200, 201], [0, 5])])
    code, msg = orc.check_image_kv(img, used, clen, head, S, keys, vals)
    assert code == 13 and "(0, 0)" in msg, msg
