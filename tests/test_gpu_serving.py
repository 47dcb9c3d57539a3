"""Serving loop: each request's result is the same served in the mix (fused
range launches per step, the step's updates fused into one call) as replayed
alone (one call per request in the same serialized order), and matches the
oracle; both sets end equal to the oracle's."""
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


def make_requests(cp, n_req, base, seed, bits=32):
    reqs = []
    kinds = synth.uniform_float(n_req, seed)
    for i in range(n_req):
        u = kinds[i]
        if u < 0.7:
            q = 1 + int(synth.uniform_keys(1, seed + 1, bits=5, offset=i)[0])
            lo = synth.uniform_keys(q, seed + 2, bits=bits, offset=64 * i)
            hi = lo + synth.uniform_keys(q, seed + 3, bits=bits - 6, offset=64 * i)
            reqs.append(cp.ServedRequest(cp.REQ_RANGE, lo, hi))
        elif u < 0.95:
            k = 1 + int(synth.uniform_keys(1, seed + 4, bits=11, offset=i)[0])
            reqs.append(cp.ServedRequest(cp.REQ_INSERT, synth.uniform_keys(k, seed + 5, bits=bits, offset=4096 * i)))
        else:
            k = 1 + int(synth.uniform_keys(1, seed + 6, bits=9, offset=i)[0])
            idx = synth.sample_indices(len(base), min(k, len(base)), seed + 7 + i)
            reqs.append(cp.ServedRequest(cp.REQ_DELETE, base[idx]))
    return reqs


@pytest.mark.parametrize("slots", [1, 16, 4096])
def test_served_equals_alone_and_oracle(cp, orc, slots):
    base = orc.build_set(synth.uniform_keys(40000, 900 + slots, bits=32))
    a = cp.CPMA(base, leaf_bytes=256)
    b = cp.CPMA(base, leaf_bytes=256)
    reqs = make_requests(cp, 400, base, 1000 + slots)
    srv = cp.Server(a, max_slots=slots)
    for r in reqs:
        srv.submit(r)
    steps = srv.stop()
    assert all(r.done for r in reqs) and all(r.req.status == 0 for r in reqs)
    if slots == 1:
        assert steps == len(reqs)
    # alone replay on b and oracle replay, in (step, ranges first, updates in arrival order)
    S = base
    order = sorted(range(len(reqs)), key=lambda i: (reqs[i].req.step, reqs[i].kind != cp.REQ_RANGE, i))
    for i in order:
        r = reqs[i]
        if r.kind == cp.REQ_RANGE:
            s1, c1 = b.range_map(r.keys, r.hi)
            s2, c2 = orc.range_map(S, r.keys, r.hi)
            assert np.array_equal(r.sum, s1) and np.array_equal(r.count, c1)
            assert np.array_equal(r.sum, s2) and np.array_equal(r.count, c2)
        elif r.kind == cp.REQ_INSERT:
            got = b.insert_batch(r.keys)
            S, added = orc.insert(S, r.keys)
            assert r.req.result == got == added
        else:
            got = b.delete_batch(r.keys)
            S, removed = orc.delete(S, r.keys)
            assert r.req.result == got == removed
    for c in (a, b):
        code, msg = orc.check_image(*c.export(), c.geometry()[1], S)
        assert code == 0, msg
        assert c.size() == len(S)


def test_serving_at_1e9_keys_properties(cp):
    """The serving benchmark's set size: 1e9 uniform 40-bit keys built on the
    GPU, then a mixed request stream through the server (inserts of fresh keys,
    deletes of present keys and of keys inserted earlier in the stream,
    re-inserts of deleted keys, ranges).  A replay by the oracle would sort 1e9
    keys on the host, so the checks are properties that hold at any size: every
    request succeeds; the set grows by exactly the added minus the removed
    counts; the full range counts the set; and every key an update touched ends
    present iff the last update on it was an insert."""
    import torch
    n = 10 ** 9
    dk = synth.uniform_keys_torch(n, synth.SEED_BASE + 2 + 70, "cuda")
    c = cp.CPMA(dk)
    n0 = c.size()
    pick = torch.from_numpy(synth.sample_indices(n, 200000, 911).astype(np.int64)).cuda()
    present = dk[pick].cpu().numpy().view(np.uint64)
    del dk, pick
    torch.cuda.empty_cache()

    kinds = synth.uniform_float(400, 912)
    sizes = synth.log_uniform_sizes(400, 913, lo_exp=1.0, hi_exp=5.0)
    reqs, inserted, deleted = [], [], []
    for i in range(400):
        m = int(sizes[i])
        if kinds[i] < 0.5:
            lo = synth.uniform_keys(4, 914 + i)
            reqs.append(cp.ServedRequest(cp.REQ_RANGE, lo, lo + np.uint64(1 << 30)))
        elif kinds[i] < 0.8:
            ks = synth.uniform_keys(m, 915 + i, offset=1 << 20)
            if deleted and i % 5 == 0:
                ks = np.concatenate([ks, deleted[-1][: m // 2]])  # re-insert deleted keys
            inserted.append(ks)
            reqs.append(cp.ServedRequest(cp.REQ_INSERT, ks))
        else:
            j = (7 * i) % (len(present) - m)
            ks = present[j:j + m]
            if inserted and i % 3 == 0:
                ks = np.concatenate([ks, inserted[-1][: m // 2]])  # delete keys inserted earlier
            deleted.append(ks)
            reqs.append(cp.ServedRequest(cp.REQ_DELETE, ks))
    srv = cp.Server(c)
    for r in reqs:
        srv.submit(r)
    srv.stop()
    assert all(r.done and r.req.status == 0 for r in reqs)
    net = sum(int(r.req.result) for r in reqs if r.kind == cp.REQ_INSERT) - \
        sum(int(r.req.result) for r in reqs if r.kind == cp.REQ_DELETE)
    assert c.size() == n0 + net
    _, cnt = c.range_map(np.array([0], np.uint64), np.array([(1 << 64) - 1], np.uint64))
    assert int(cnt[0]) == c.size()
    # final membership of every touched key: the last update on it decides
    # (the server applies updates in arrival order)
    ups = [(r.keys, 1 if r.kind == cp.REQ_INSERT else 0) for r in reqs if r.kind != cp.REQ_RANGE]
    keys = np.concatenate([k for k, _ in ups])
    state = np.concatenate([np.full(len(k), s, np.uint8) for k, s in ups])
    order = np.arange(len(keys))
    srt = np.lexsort((order, keys))
    keys, state = keys[srt], state[srt]
    last = np.r_[keys[1:] != keys[:-1], True]
    assert np.array_equal(c.contains(keys[last]), state[last])
