"""cpma_range_map_noalloc: the range_map entry point that allocates nothing,
checked through the C ABI against cpma_range_map (the entry point it mirrors)
and the oracle, on two calls in a row, the second with fewer queries."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_noalloc_range_map_matches_range_map(orc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_05055_amd as cp
    L = cp.lib()
    ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
    FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
    calls = [0]
    live = {}

    def _alloc(n, ctx):
        calls[0] += 1
        p = torch.cuda.caching_allocator_alloc(n)
        live[p] = n
        return p

    def _free(p, ctx):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    a_cb, f_cb = ALLOC(_alloc), FREE(_free)
    cfg = cp.default_config()
    cfg.alloc = ctypes.cast(a_cb, ctypes.c_void_p).value
    cfg.free = ctypes.cast(f_cb, ctypes.c_void_p).value
    keys = synth.uniform_keys(300000, 4401, bits=40)
    expect = orc.build_set(keys)
    c = cp.CPMA(keys, config=cfg)

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64)).cuda()

    st = torch.cuda.current_stream()
    for q, width, seed in ((cp.NOALLOC_MAX_QUERIES, 1 << 30, 4402), (777, 1 << 34, 4403)):
        lo, hi = synth.range_queries_width(q, seed, width)
        lo[:5] = hi[:5]                            # empty ranges
        lo[5], hi[5] = 0, (1 << 64) - 1            # the whole key space
        dlo, dhi = dev(lo), dev(hi)
        s_ref, n_ref = c.range_map(dlo, dhi)       # the existing entry point
        s_out = torch.full((q,), -1, dtype=torch.int64, device="cuda")
        n_out = torch.full((q,), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        before = calls[0]
        r = L.cpma_range_map_noalloc(c._h, ctypes.c_void_p(dlo.data_ptr()), ctypes.c_void_p(dhi.data_ptr()), q,
                                     ctypes.c_void_p(s_out.data_ptr()), ctypes.c_void_p(n_out.data_ptr()),
                                     ctypes.c_void_p(st.cuda_stream))
        assert r == 0
        torch.cuda.synchronize()
        assert calls[0] == before                  # nothing taken from the allocator
        assert torch.equal(s_out, s_ref) and torch.equal(n_out, n_ref)
        es, en = orc.range_map(expect, lo, hi)
        assert np.array_equal(s_out.cpu().numpy().view(np.uint64), es)
        assert np.array_equal(n_out.cpu().numpy().view(np.uint64), en)
    # beyond the fixed scratch: rejected before anything is launched
    big = cp.NOALLOC_MAX_QUERIES + 1
    z = torch.zeros(big, dtype=torch.int64, device="cuda")
    assert L.cpma_range_map_noalloc(c._h, ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()), big,
                                    ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                    ctypes.c_void_p(st.cuda_stream)) == 1
    # the binding's wrapper gives the same
    s2, n2 = c.range_map_noalloc(dlo, dhi)
    torch.cuda.synchronize()
    assert torch.equal(s2, s_ref) and torch.equal(n2, n_ref)
    c.close()
    assert not live
