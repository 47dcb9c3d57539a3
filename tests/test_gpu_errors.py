"""Error contract of an update (the boundary's rule: an error leaves the set
unchanged): an allocator that stops giving memory at any point of an update
either leaves the set exactly as it was (CPMA_ERR_NOMEM, handle still usable)
or the update completes without the memory it was refused.  Every allocation
point of an update is tried in turn."""
import ctypes

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


class Hooks:
    """Device allocator hooks over torch's caching allocator that refuse every
    request from the fail_from-th call on."""

    def __init__(self, cp):
        import torch
        self.torch = torch
        self.calls = 0
        self.refused = 0
        self.fail_from = None
        self.live = {}
        ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
        FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
        self._a = ALLOC(self.alloc)
        self._f = FREE(self.free)
        self.cfg = cp.default_config()
        self.cfg.alloc = ctypes.cast(self._a, ctypes.c_void_p).value
        self.cfg.free = ctypes.cast(self._f, ctypes.c_void_p).value

    def alloc(self, n, ctx):
        self.calls += 1
        if self.fail_from is not None and self.calls >= self.fail_from:
            self.refused += 1
            return None
        p = self.torch.cuda.caching_allocator_alloc(n)
        self.live[p] = n
        return p

    def free(self, p, ctx):
        self.live.pop(p)
        self.torch.cuda.caching_allocator_delete(p)


def _image(c):
    b, u, h = c.export()
    return b.copy(), u.copy(), h.copy()


def _check(c, expect, orc):
    b, u, h = c.export()
    L, S = c.geometry()
    code, msg = orc.check_image(b, u, h, S, expect)
    assert code == 0, msg
    assert c.size() == len(expect)


def _sweep(cp, orc, base, batch, S, insert, after):
    """Refuses memory from each allocation call of the update on; returns the
    number of trials that completed although memory was refused."""
    hk = Hooks(cp)
    hk.cfg.leaf_bytes = S
    # a reference run counts the update's allocation calls
    c = cp.CPMA(base, config=hk.cfg)
    start = hk.calls
    (c.insert_batch if insert else c.delete_batch)(batch)
    n_calls = hk.calls - start
    c.close()
    assert not hk.live
    expect0 = orc.build_set(base)
    expect1 = orc.insert(expect0, batch)[0] if insert else orc.delete(expect0, batch)[0]
    completed_refused = 0
    for j in range(n_calls + 1):
        hk.fail_from = None
        c = cp.CPMA(base, config=hk.cfg)
        before = _image(c)
        hk.refused = 0
        hk.fail_from = hk.calls + 1 + j
        try:
            (c.insert_batch if insert else c.delete_batch)(batch)
            ok = True
        except cp.CpmaError as e:
            assert e.code == 2, f"allocation {j}: status {e.code}, not CPMA_ERR_NOMEM"
            ok = False
        hk.fail_from = None
        if ok:
            _check(c, expect1, orc)
            completed_refused += hk.refused > 0
        else:
            after_img = _image(c)
            assert all(np.array_equal(x, y) for x, y in zip(before, after_img)), f"allocation {j}: set changed"
            _check(c, expect0, orc)
            # the handle is still usable: the same update now succeeds
            (c.insert_batch if insert else c.delete_batch)(batch)
            _check(c, expect1, orc)
        # and so does the next one
        e2, added = orc.insert(expect1, after)
        assert c.insert_batch(after) == added
        _check(c, e2, orc)
        c.close()
        assert not hk.live
    return n_calls, completed_refused


def test_nomem_at_every_allocation_of_a_growing_insert(cp, orc):
    base = synth.uniform_keys(60000, 9101, bits=40)
    batch = synth.uniform_keys(60000, 9102, bits=40)   # doubles the set: grows
    after = synth.uniform_keys(500, 9103, bits=40)
    n_calls, _ = _sweep(cp, orc, base, batch, 256, True, after)
    assert n_calls > 0


def test_nomem_at_every_allocation_of_a_small_batch(cp, orc):
    base = synth.uniform_keys(60000, 9111, bits=40)
    batch = synth.uniform_keys(300, 9112, bits=40)      # the one-launch preparation path
    after = synth.uniform_keys(500, 9113, bits=40)
    _sweep(cp, orc, base, batch, 256, True, after)


def test_nomem_at_every_allocation_of_a_delete(cp, orc):
    base = synth.uniform_keys(60000, 9121, bits=40)
    expect = orc.build_set(base)
    batch = expect[synth.sample_indices(len(expect), 45000, 9122)]   # shrinks
    after = synth.uniform_keys(500, 9123, bits=40)
    _sweep(cp, orc, base, batch, 256, False, after)


def test_nomem_in_redistribution_falls_back_to_a_full_spread(cp, orc):
    """A batch packed into one narrow key range overfills a few leaves, so the
    update redistributes windows without growing.  Refused staging memory for
    the windows makes it spread the whole structure instead (with memory taken
    before the merge): some trials complete although memory was refused."""
    base = synth.uniform_keys(200000, 9131, bits=40)
    x0 = np.uint64(1 << 39)
    batch = x0 + synth.uniform_keys(3000, 9132, bits=24)
    after = synth.uniform_keys(500, 9133, bits=40)
    n_calls, completed = _sweep(cp, orc, base, batch, 256, True, after)
    assert completed > 0, "no trial took the full-spread fallback"


def test_bytes_held_counts_spares_and_scratch(cp, orc):
    c = cp.CPMA(synth.uniform_keys(100000, 9141, bits=40))
    c.insert_batch(synth.uniform_keys(50000, 9142, bits=40))
    assert c.bytes_held() > c.bytes()
    c.close()


def test_trim_releases_scratch_and_later_calls_still_agree(cp, orc):
    """After a large batch the handle keeps that batch's scratch; trim releases
    everything but the structure and a few counters, and later updates and
    queries (which allocate again) still match the oracle."""
    base = synth.uniform_keys(200000, 9151, bits=40)
    ins = synth.uniform_keys(150000, 9152, bits=40)
    c = cp.CPMA(base)
    c.insert_batch(ins)
    held = c.bytes_held()
    assert held > 2 * c.bytes()
    c.trim()
    assert c.bytes_held() <= c.bytes() + 4096
    assert c.bytes_held() < held
    ref = orc.insert(orc.build_set(base), ins)[0]
    dels = ins[::3]
    assert c.delete_batch(dels) == len(np.unique(dels))
    ref = orc.delete(ref, dels)[0]
    more = synth.uniform_keys(30000, 9153, bits=40)
    c.insert_batch(more)
    ref = orc.insert(ref, more)[0]
    c.trim()
    b, u, h = c.export()
    code, msg = orc.check_image(b, u, h, c.geometry()[1], ref)
    assert code == 0, msg
    lo = np.array([0, ref[100]], np.uint64)
    hi = np.array([np.uint64(1) << np.uint64(40), ref[5000]], np.uint64)
    s, n = c.range_map(lo, hi)
    es, en = orc.range_map(ref, lo, hi)
    assert np.array_equal(s, es) and np.array_equal(n, en)
    c.close()
