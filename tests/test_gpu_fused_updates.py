"""Fused application of a request sequence (cpma_apply_updates) against the
oracle replaying the requests one call each, in order: every request's count is
bit-exact and the final set passes the structure checker against the oracle's
set.  Key domains are small so that requests share keys, and requests repeat
keys, so that a key's occurrences span several requests of both kinds."""
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


def replay(orc, cp, S, reqs):
    counts = []
    for kind, keys in reqs:
        if kind == cp.REQ_INSERT:
            S, c = orc.insert(S, keys)
        else:
            S, c = orc.delete(S, keys)
        counts.append(c)
    return S, counts


def check(c, expect, orc):
    b, u, h = c.export()
    code, msg = orc.check_image(b, u, h, c.geometry()[1], expect)
    assert code == 0, msg
    assert c.size() == len(expect)


def mixed_requests(cp, nreq, seed, bits, max_len, del_frac=0.4):
    kinds = synth.uniform_float(nreq, seed)
    lens = synth.uniform_keys(nreq, seed + 1, bits=max_len.bit_length() + 1) % (max_len + 1)
    out = []
    for i in range(nreq):
        keys = synth.uniform_keys(int(lens[i]), seed + 2 + i, bits=bits)
        out.append((cp.REQ_DELETE if kinds[i] < del_frac else cp.REQ_INSERT, keys))
    return out


@pytest.mark.parametrize("seed,nreq,bits,max_len,n0", [
    (1, 40, 12, 300, 2000),      # tiny domain: every key in many requests
    (2, 200, 16, 200, 20000),    # small net batches (one-launch prep path)
    (3, 30, 24, 40000, 100000),  # large net batches (radix-sorted path)
    (4, 1, 20, 50000, 50000),    # a single request
])
def test_fused_matches_sequential_replay(cp, orc, seed, nreq, bits, max_len, n0):
    base = orc.build_set(synth.uniform_keys(n0, 100 + seed, bits=bits))
    reqs = mixed_requests(cp, nreq, 200 + seed, bits, max_len)
    c = cp.CPMA(base, leaf_bytes=256)
    got = c.apply_updates(reqs)
    S, want = replay(orc, cp, base, reqs)
    assert got == want
    check(c, S, orc)


def test_one_key_alternating_and_repeats(cp, orc):
    # one key inserted and deleted in turn across 501 requests, with repeats
    # inside requests and empty requests between them
    base = orc.build_set(synth.uniform_keys(5000, 11, bits=20))
    x = np.array([int(base[17])], np.uint64)          # present at the start
    y = np.array([(1 << 20) + 5], np.uint64)          # absent at the start
    reqs = []
    for i in range(501):
        kind = cp.REQ_DELETE if i % 2 == 0 else cp.REQ_INSERT
        reqs.append((kind, np.concatenate([x, x, y] if i % 3 else [x])))
        if i % 7 == 0:
            reqs.append((cp.REQ_INSERT, np.empty(0, np.uint64)))
    c = cp.CPMA(base, leaf_bytes=256)
    got = c.apply_updates(reqs)
    S, want = replay(orc, cp, base, reqs)
    assert got == want
    check(c, S, orc)


def test_growth_then_shrink_in_one_call(cp, orc):
    # net inserts that grow the array several times, then net deletes of most
    # keys in a second call (shrink)
    base = orc.build_set(synth.uniform_keys(3000, 21, bits=40))
    new = synth.uniform_keys(300000, 22, bits=40)
    reqs = [(cp.REQ_INSERT, new[i::7]) for i in range(7)] + [(cp.REQ_DELETE, base[::3])]
    c = cp.CPMA(base, leaf_bytes=128)
    L0 = c.geometry()[0]
    got = c.apply_updates(reqs)
    S, want = replay(orc, cp, base, reqs)
    assert got == want
    check(c, S, orc)
    assert c.geometry()[0] > L0
    reqs2 = [(cp.REQ_DELETE, S[i::5]) for i in range(4)] + [(cp.REQ_INSERT, S[:10])]
    got2 = c.apply_updates(reqs2)
    S2, want2 = replay(orc, cp, S, reqs2)
    assert got2 == want2
    check(c, S2, orc)


def test_empty_sequences_and_no_net_change(cp, orc):
    base = orc.build_set(synth.uniform_keys(4000, 31, bits=24))
    c = cp.CPMA(base, leaf_bytes=256)
    assert c.apply_updates([]) == []
    assert c.apply_updates([(cp.REQ_INSERT, np.empty(0, np.uint64))] * 3) == [0, 0, 0]
    # insert then delete the same absent keys: counts but no net change
    fresh = np.setdiff1d(synth.uniform_keys(500, 32, bits=24), base)
    got = c.apply_updates([(cp.REQ_INSERT, fresh), (cp.REQ_DELETE, fresh), (cp.REQ_INSERT, base[:50])])
    assert got == [len(fresh), len(fresh), 0]
    check(c, base, orc)


def test_reserved_key_and_bad_tables_change_nothing(cp, orc):
    base = orc.build_set(synth.uniform_keys(2000, 41, bits=32))
    c = cp.CPMA(base, leaf_bytes=256)
    with pytest.raises(cp.CpmaError) as e:
        c.apply_updates([(cp.REQ_INSERT, np.array([1, 2], np.uint64)),
                         (cp.REQ_DELETE, np.array([3, M64], np.uint64))])
    assert e.value.code == 4
    with pytest.raises(cp.CpmaError) as e:
        c.apply_updates([(cp.REQ_RANGE, np.array([1], np.uint64))])
    assert e.value.code == 1
    check(c, base, orc)
    # the set still works afterwards
    assert c.apply_updates([(cp.REQ_INSERT, np.array([7], np.uint64))]) == [0 if 7 in set(base.tolist()) else 1]


def test_device_resident_requests(cp, orc):
    import torch
    base = orc.build_set(synth.uniform_keys(30000, 51, bits=22))
    host = mixed_requests(cp, 60, 52, 22, 3000)
    dev = [(k, torch.from_numpy(ks.view(np.int64)).cuda()) for k, ks in host]
    c = cp.CPMA(base, leaf_bytes=512)
    got = c.apply_updates(dev)
    S, want = replay(orc, cp, base, host)
    assert got == want
    check(c, S, orc)


def test_mixed_direct_and_packed_host_copies(cp, orc):
    # requests above and below the direct-copy size interleaved, so packed runs
    # of small requests sit between directly copied large ones
    base = orc.build_set(synth.uniform_keys(50000, 61, bits=30))
    reqs = []
    for i in range(12):
        n = 40000 if i % 3 == 0 else 1 + 37 * i
        reqs.append((cp.REQ_DELETE if i % 4 == 1 else cp.REQ_INSERT, synth.uniform_keys(n, 62 + i, bits=30)))
    c = cp.CPMA(base, leaf_bytes=1024)
    got = c.apply_updates(reqs)
    S, want = replay(orc, cp, base, reqs)
    assert got == want
    check(c, S, orc)
