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
    S = replay_and_check(cp, orc, reqs, base, b)
    for c in (a, b):
        code, msg = orc.check_image(*c.export(), c.geometry()[1], S)
        assert code == 0, msg
        assert c.size() == len(S)


def replay_and_check(cp, orc, reqs, S0, b=None):
    """Checks every served result against two replays and returns the oracle's
    final set.

    * The server's order -- by step, a step's ranges before its updates, updates
      in arrival order -- replayed one call per request on the set b (when
      given) and by the oracle: every result must be equal.
    * Pure arrival order, by the oracle: every update's result and every range
      that no update of its own step preceded must be equal too; a range that
      arrived after an update of its own step sees the state at the start of
      its step instead (the documented step semantics, checked above)."""
    S = S0
    order = sorted(range(len(reqs)), key=lambda i: (reqs[i].req.step, reqs[i].kind != cp.REQ_RANGE, i))
    for i in order:
        r = reqs[i]
        if r.kind == cp.REQ_RANGE:
            s2, c2 = orc.range_map(S, r.keys, r.hi)
            assert np.array_equal(r.sum, s2) and np.array_equal(r.count, c2), i
            if b is not None:
                s1, c1 = b.range_map(r.keys, r.hi)
                assert np.array_equal(r.sum, s1) and np.array_equal(r.count, c1), i
        elif r.kind == cp.REQ_INSERT:
            S, added = orc.insert(S, r.keys)
            assert r.req.result == added, i
            if b is not None:
                assert b.insert_batch(r.keys) == added, i
        else:
            S, removed = orc.delete(S, r.keys)
            assert r.req.result == removed, i
            if b is not None:
                assert b.delete_batch(r.keys) == removed, i
    A = S0
    update_seen = set()
    reordered = 0
    for i, r in enumerate(reqs):
        step = r.req.step
        if r.kind == cp.REQ_RANGE:
            if step in update_seen:
                reordered += 1
                continue
            s2, c2 = orc.range_map(A, r.keys, r.hi)
            assert np.array_equal(r.sum, s2) and np.array_equal(r.count, c2), i
        else:
            update_seen.add(step)
            if r.kind == cp.REQ_INSERT:
                A, x = orc.insert(A, r.keys)
            else:
                A, x = orc.delete(A, r.keys)
            assert r.req.result == x, i
    assert np.array_equal(A, S)
    return S


def config5_requests(cp, n_req, n0, seed, base_at, lmax=10 ** 5, size_hi_exp=6.0):
    """A request stream shaped like the serving benchmark's: 70 % range requests
    (one range of Zipf(1.2) length on 1..lmax keys, width length * floor(2^40 /
    n0), lo uniform), 25 % inserts of fresh uniform 40-bit keys and 5 % deletes
    of keys of the initial set, update sizes floor(10^(1 + 5u))-like log-uniform
    from 10 up to 10^size_hi_exp.  base_at(indices) gives initial keys."""
    width = (1 << 40) // n0
    kinds = synth.uniform_float(n_req, seed)
    lens = synth.zipf_lengths(n_req, seed + 1, alpha=1.2, lmax=lmax)
    sizes = synth.log_uniform_sizes(n_req, seed + 2, lo_exp=1.0, hi_exp=size_hi_exp)
    los = synth.uniform_keys(n_req, seed + 3)
    reqs = []
    for i in range(n_req):
        if kinds[i] < 0.70:
            lo = los[i:i + 1]
            reqs.append(cp.ServedRequest(cp.REQ_RANGE, lo, lo + np.uint64(int(lens[i]) * width)))
        elif kinds[i] < 0.95:
            reqs.append(cp.ServedRequest(cp.REQ_INSERT, synth.uniform_keys(int(sizes[i]), seed + 4,
                                                                           offset=10 ** 7 * i)))
        else:
            idx = synth.sample_indices(n0, int(sizes[i]), seed + 5 + i)
            reqs.append(cp.ServedRequest(cp.REQ_DELETE, base_at(idx)))
    return reqs


def serve(cp, c, reqs, slots=4096):
    srv = cp.Server(c, max_slots=slots)
    for r in reqs:
        srv.submit(r)
    steps = srv.stop()
    assert all(r.done and r.req.status == 0 for r in reqs)
    return steps


def test_config5_stream_exact_at_1e7(cp, orc):
    """The serving benchmark's request shapes (Zipf range lengths up to 1e5 keys,
    updates up to 1e6 keys) on a set of 1e7 uniform 40-bit keys, replayed
    exactly: served, alone and by the oracle."""
    import torch
    n0 = 10 ** 7
    seed = synth.SEED_BASE + 805
    keys = synth.uniform_keys(n0, seed)
    base = orc.build_set(keys)
    dk = torch.from_numpy(keys.view(np.int64)).cuda()
    a, b = cp.CPMA(dk), cp.CPMA(dk)
    del dk
    reqs = config5_requests(cp, 240, n0, seed + 10, lambda idx: keys[idx])
    assert sum(r.kind == cp.REQ_INSERT and len(r.keys) > 10 ** 5 for r in reqs) > 0
    steps = serve(cp, a, reqs)
    assert steps >= 1
    S = replay_and_check(cp, orc, reqs, base, b)
    for c in (a, b):
        code, msg = orc.check_image(*c.export(), c.geometry()[1], S)
        assert code == 0, msg


def test_config5_prefix_exact_at_1e9(cp, orc):
    """The serving benchmark's set itself (1e9 uniform 40-bit keys) and a prefix
    of 300 requests of its stream, replayed exactly.  The oracle does not need
    all 1e9 keys: every result depends only on the keys inside the requests'
    ranges and on the membership of the requests' update keys.  The keys of
    the generated stream that fall in that universe are selected with torch
    (the stream's torch twin and torch's own searchsorted; nothing of this
    library), and the oracle replays the requests on them: range sums and
    counts, n_added and n_removed are all exact.  Served results must equal it
    and an alone replay on a second 1e9-key set."""
    import torch
    n = 10 ** 9
    seed = synth.SEED_BASE + 2 + 70
    reqs = config5_requests(cp, 300, n, synth.SEED_BASE + 906, lambda idx: synth.uniform_keys_at(idx, seed),
                            size_hi_exp=5.5)
    ranges = [(int(r.keys[0]), int(r.hi[0])) for r in reqs if r.kind == cp.REQ_RANGE]
    pts = np.unique(np.concatenate([r.keys for r in reqs if r.kind != cp.REQ_RANGE]))
    # merge the ranges into disjoint intervals
    ranges.sort()
    iv = []
    for lo, hi in ranges:
        if iv and lo <= iv[-1][1]:
            iv[-1][1] = max(iv[-1][1], hi)
        else:
            iv.append([lo, hi])
    st = torch.tensor([x[0] for x in iv], dtype=torch.int64, device="cuda")
    en = torch.tensor([x[1] for x in iv], dtype=torch.int64, device="cuda")   # 40-bit keys: no sign issue
    pt = torch.from_numpy(pts.view(np.int64)).cuda()
    dk = synth.uniform_keys_torch(n, seed, "cuda")
    sel = []
    for o in range(0, n, 1 << 27):
        x = dk[o:o + (1 << 27)]
        i = torch.searchsorted(st, x, right=True) - 1
        inside = (i >= 0) & (x < en[i.clamp(min=0)])
        j = torch.searchsorted(pt, x).clamp(max=len(pt) - 1)
        sel.append(x[inside | (pt[j] == x)].cpu())
    R0 = orc.build_set(torch.cat(sel).numpy().view(np.uint64))
    a = cp.CPMA(dk)
    b = cp.CPMA(dk)
    n0 = a.size()
    del dk, x, i, inside, j
    torch.cuda.empty_cache()
    serve(cp, a, reqs)
    S = replay_and_check(cp, orc, reqs, R0, b)
    net = sum(int(r.req.result) for r in reqs if r.kind == cp.REQ_INSERT) - \
        sum(int(r.req.result) for r in reqs if r.kind == cp.REQ_DELETE)
    assert a.size() == b.size() == n0 + net
    _, cnt = a.range_map(np.array([0], np.uint64), np.array([(1 << 64) - 1], np.uint64))
    assert int(cnt[0]) == a.size()
    # every updated key ends present or absent as the oracle says
    assert np.array_equal(a.contains(pts), orc.contains(S, pts))


def test_batched_range_map_equals_one_launch_per_query(cp, orc):
    """Zipf(1.2) exact-count queries on a 1e7-key set: one launch for all of them,
    one launch per query and the oracle agree."""
    import torch
    keys = synth.unique_uniform_keys(10 ** 7, synth.SEED_BASE + 811)
    S = orc.build_set(keys)
    c = cp.CPMA(keys)
    lens = synth.zipf_lengths(2000, synth.SEED_BASE + 812, alpha=1.2, lmax=10 ** 6)
    lo, hi = synth.range_queries_by_count(S, lens, synth.SEED_BASE + 813)
    dlo = torch.from_numpy(lo.view(np.int64)).cuda()
    dhi = torch.from_numpy(hi.view(np.int64)).cuda()
    bs, bn = c.range_map(dlo, dhi)
    one = [c.range_map(dlo[i:i + 1], dhi[i:i + 1]) for i in range(len(lo))]
    os_ = torch.cat([x[0] for x in one])
    on = torch.cat([x[1] for x in one])
    assert torch.equal(bs, os_) and torch.equal(bn, on)
    es, en = orc.range_map(S, lo, hi)
    assert np.array_equal(bs.cpu().numpy().view(np.uint64), es)
    assert np.array_equal(bn.cpu().numpy().view(np.uint64), en)
    assert np.array_equal(en, np.minimum(lens, len(S)).astype(np.uint64))


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


def test_requests_admitted_while_a_step_runs(cp, orc):
    """Continuous batching: requests that arrive while a step is on the GPU are
    admitted (and their data uploaded) before that step ends, then served in
    the next step; results still equal the replays."""
    import time
    base = orc.build_set(synth.uniform_keys(400000, 9301, bits=40))
    a = cp.CPMA(base, leaf_bytes=256)
    b = cp.CPMA(base, leaf_bytes=256)
    reqs = []
    kinds = synth.uniform_float(240, 9302)
    for i in range(240):
        if kinds[i] < 0.6:
            lo = synth.uniform_keys(8, 9303, offset=8 * i)
            reqs.append(cp.ServedRequest(cp.REQ_RANGE, lo, lo + np.uint64(1 << 28)))
        elif kinds[i] < 0.9:
            reqs.append(cp.ServedRequest(cp.REQ_INSERT, synth.uniform_keys(30000, 9304, offset=30000 * i)))
        else:
            idx = synth.sample_indices(len(base), 5000, 9305 + i)
            reqs.append(cp.ServedRequest(cp.REQ_DELETE, base[idx]))
    srv = cp.Server(a)
    for r in reqs:
        srv.submit(r)
        t_end = time.perf_counter() + 200e-6   # a request every 200 us
        while time.perf_counter() < t_end:
            pass
    steps = srv.stop()
    assert all(r.done and r.req.status == 0 for r in reqs)
    assert steps > 2
    ends = {}
    for r in reqs:
        ends[r.req.step] = max(ends.get(r.req.step, 0), r.req.t_done_ns)
    early = sum(1 for r in reqs if r.req.step > 0 and r.req.t_admit_ns < ends[r.req.step - 1])
    assert early > 0, "no request was admitted while the step before it ran"
    assert all(r.req.t_admit_ns >= r.t_submit_ns and r.req.t_done_ns >= r.req.t_admit_ns for r in reqs)
    S = replay_and_check(cp, orc, reqs, base, b)
    code, msg = orc.check_image(*a.export(), a.geometry()[1], S)
    assert code == 0, msg
