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
