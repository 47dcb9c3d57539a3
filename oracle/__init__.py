"""CPU oracle for the CPMA hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library under ``paper_2305_05055_amd``) never touches it.

The C++ source (``oracle.cpp``) is the plain definition of what the CPMA
computes (an exact ordered set of 64-bit keys; Section "Packed Memory Array",
"Design and operations", and the appendix "PMA/CPMA API"), an independent
LEB128 byte-code codec (Section "Compressed Packed Memory Array", "Data
compression techniques"), a structure checker for the leaf layout and the
density bounds of the implicit tree, and FP64 PageRank / BFS over edge keys
``src<<32|dst`` (Section "Evaluation on graph workloads").
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

# Default density-bound parameters {up_leaf, up_root, lo_leaf, lo_root}.
DEFAULT_PARAMS = (0.90, 0.70, 0.10, 0.30)


def build(force=True):
    """Compile liboracle.so with g++ (plain C++17, no GPU code)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        dp = ctypes.POINTER(ctypes.c_double)
        c_u64 = ctypes.c_uint64
        L.orc_build.argtypes = [u64p, c_u64, u64p]
        L.orc_build.restype = c_u64
        L.orc_insert.argtypes = [u64p, c_u64, u64p, c_u64, u64p, u64p]
        L.orc_insert.restype = c_u64
        L.orc_delete.argtypes = [u64p, c_u64, u64p, c_u64, u64p, u64p]
        L.orc_delete.restype = c_u64
        L.orc_contains.argtypes = [u64p, c_u64, u64p, c_u64, u8p]
        L.orc_range_map.argtypes = [u64p, c_u64, u64p, u64p, c_u64, u64p, u64p]
        L.orc_range_map_threads.argtypes = [u64p, c_u64, u64p, u64p, c_u64, u64p, u64p, ctypes.c_int]
        L.orc_range_map_brute.argtypes = [u64p, c_u64, u64p, u64p, c_u64, u64p, u64p]
        L.orc_varint_encode.argtypes = [c_u64, u8p]
        L.orc_varint_encode.restype = ctypes.c_int
        L.orc_varint_decode.argtypes = [u8p, ctypes.c_int, u64p]
        L.orc_varint_decode.restype = ctypes.c_int
        L.orc_bound_q.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_bound_q.restype = ctypes.c_int64
        L.orc_tree_height.argtypes = [c_u64]
        L.orc_tree_height.restype = ctypes.c_int
        L.orc_check_image.argtypes = [u8p, u32p, u64p, c_u64, ctypes.c_uint32, dp, u64p,
                                      c_u64, ctypes.c_char_p, ctypes.c_int]
        L.orc_check_image.restype = ctypes.c_int
        L.orc_check_image_pma.argtypes = L.orc_check_image.argtypes
        L.orc_check_image_pma.restype = ctypes.c_int
        L.orc_check_image_kv.argtypes = [u8p, u32p, u32p, u64p, c_u64, ctypes.c_uint32, dp, u64p, u64p,
                                         c_u64, ctypes.c_char_p, ctypes.c_int]
        L.orc_check_image_kv.restype = ctypes.c_int
        L.orc_decode_image.argtypes = [u8p, u32p, c_u64, ctypes.c_uint32, u64p, c_u64]
        L.orc_decode_image.restype = ctypes.c_int64
        L.orc_bfs.argtypes = [u64p, c_u64, ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.orc_offsets.argtypes = [u64p, c_u64, ctypes.c_uint32, u64p]
        L.orc_cc.argtypes = [u64p, c_u64, ctypes.c_uint32, u32p]
        L.orc_bc.argtypes = [u64p, c_u64, ctypes.c_uint32, ctypes.c_uint32, dp, dp]
        L.orc_pagerank.argtypes = [u64p, c_u64, ctypes.c_uint32, ctypes.c_int,
                                   ctypes.c_double, dp]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def build_set(keys):
    k = _u64(keys)
    out = np.empty(len(k), dtype=np.uint64)
    m = lib().orc_build(_p(k, ctypes.c_uint64), len(k), _p(out, ctypes.c_uint64))
    return out[:m].copy()


def insert(S, B):
    S, B = _u64(S), _u64(B)
    out = np.empty(len(S) + len(B), dtype=np.uint64)
    added = ctypes.c_uint64(0)
    m = lib().orc_insert(_p(S, ctypes.c_uint64), len(S), _p(B, ctypes.c_uint64), len(B),
                         _p(out, ctypes.c_uint64), ctypes.byref(added))
    return out[:m].copy(), int(added.value)


def delete(S, B):
    S, B = _u64(S), _u64(B)
    out = np.empty(len(S), dtype=np.uint64)
    removed = ctypes.c_uint64(0)
    m = lib().orc_delete(_p(S, ctypes.c_uint64), len(S), _p(B, ctypes.c_uint64), len(B),
                         _p(out, ctypes.c_uint64), ctypes.byref(removed))
    return out[:m].copy(), int(removed.value)


def contains(S, q):
    S, q = _u64(S), _u64(q)
    out = np.empty(len(q), dtype=np.uint8)
    lib().orc_contains(_p(S, ctypes.c_uint64), len(S), _p(q, ctypes.c_uint64), len(q),
                       _p(out, ctypes.c_uint8))
    return out


def range_map(S, lo, hi, brute=False, threads=0):
    """threads > 0: the queries split over that many host threads."""
    S, lo, hi = _u64(S), _u64(lo), _u64(hi)
    s = np.empty(len(lo), dtype=np.uint64)
    c = np.empty(len(lo), dtype=np.uint64)
    args = (_p(S, ctypes.c_uint64), len(S), _p(lo, ctypes.c_uint64), _p(hi, ctypes.c_uint64),
            len(lo), _p(s, ctypes.c_uint64), _p(c, ctypes.c_uint64))
    if threads > 0:
        lib().orc_range_map_threads(*args, int(threads))
    else:
        (lib().orc_range_map_brute if brute else lib().orc_range_map)(*args)
    return s, c


def varint_encode(x):
    buf = (ctypes.c_uint8 * 16)()
    n = lib().orc_varint_encode(ctypes.c_uint64(int(x)), buf)
    return bytes(buf[:n])


def varint_decode(b):
    arr = (ctypes.c_uint8 * max(1, len(b)))(*b)
    x = ctypes.c_uint64(0)
    n = lib().orc_varint_decode(arr, len(b), ctypes.byref(x))
    return (int(x.value), n) if n >= 0 else (None, n)


def bound_q(which, h, H, params=DEFAULT_PARAMS):
    pa = (ctypes.c_double * 4)(*params)
    return int(lib().orc_bound_q(pa, which, h, H))


def tree_height(L):
    return int(lib().orc_tree_height(int(L)))


def check_image(bytes_, used, head, S, expect, params=DEFAULT_PARAMS):
    """Returns (code, message); code 0 means every invariant holds."""
    b = np.ascontiguousarray(bytes_, dtype=np.uint8)
    u = np.ascontiguousarray(used, dtype=np.uint32)
    h = _u64(head)
    e = _u64(expect)
    L = len(u)
    assert len(b) == L * S and len(h) == L
    pa = (ctypes.c_double * 4)(*params)
    msg = ctypes.create_string_buffer(256)
    code = lib().orc_check_image(_p(b, ctypes.c_uint8), _p(u, ctypes.c_uint32),
                                 _p(h, ctypes.c_uint64), L, S, pa, _p(e, ctypes.c_uint64),
                                 len(e), msg, 256)
    return int(code), msg.value.decode()


def check_image_pma(bytes_, used, head, S, expect, params=DEFAULT_PARAMS):
    """check_image for the uncompressed variant (raw 8-byte keys per leaf)."""
    b = np.ascontiguousarray(bytes_, dtype=np.uint8)
    u = np.ascontiguousarray(used, dtype=np.uint32)
    h = _u64(head)
    e = _u64(expect)
    L = len(u)
    assert len(b) == L * S and len(h) == L
    pa = (ctypes.c_double * 4)(*params)
    msg = ctypes.create_string_buffer(256)
    code = lib().orc_check_image_pma(_p(b, ctypes.c_uint8), _p(u, ctypes.c_uint32),
                                     _p(h, ctypes.c_uint64), L, S, pa, _p(e, ctypes.c_uint64),
                                     len(e), msg, 256)
    return int(code), msg.value.decode()


def check_image_kv(bytes_, used, clen, head, S, expect, expect_vals, params=DEFAULT_PARAMS):
    """check_image for key-value leaves (codes, then values at the leaf's end)."""
    b = np.ascontiguousarray(bytes_, dtype=np.uint8)
    u = np.ascontiguousarray(used, dtype=np.uint32)
    c = np.ascontiguousarray(clen, dtype=np.uint32)
    h = _u64(head)
    e = _u64(expect)
    ev = _u64(expect_vals)
    L = len(u)
    assert len(b) == L * S and len(h) == L and len(c) == L and len(ev) == len(e)
    pa = (ctypes.c_double * 4)(*params)
    msg = ctypes.create_string_buffer(256)
    code = lib().orc_check_image_kv(_p(b, ctypes.c_uint8), _p(u, ctypes.c_uint32), _p(c, ctypes.c_uint32),
                                    _p(h, ctypes.c_uint64), L, S, pa, _p(e, ctypes.c_uint64),
                                    _p(ev, ctypes.c_uint64), len(e), msg, 256)
    return int(code), msg.value.decode()


# ---- the key-value set (sorted keys with their values) -----------------------------
# A key-value set is a pair (K, V): K the sorted distinct keys, V[i] the value
# of K[i].  Batches may repeat a key; its first occurrence counts.

def kv_build(keys, vals):
    k = _u64(keys)
    v = _u64(vals)
    K, first = np.unique(k, return_index=True)
    return K, v[first].copy()


def kv_insert(K, V, keys, vals):
    """Upsert: new keys join with their values, present keys take the new
    value.  Returns (K', V', number of keys added)."""
    bk, bv = kv_build(keys, vals)
    pos = np.searchsorted(K, bk)
    present = (pos < len(K)) & (K[np.minimum(pos, max(len(K) - 1, 0))] == bk) if len(K) else np.zeros(len(bk), bool)
    V2 = V.copy()
    V2[pos[present]] = bv[present]
    nk = np.concatenate([K, bk[~present]])
    nv = np.concatenate([V2, bv[~present]])
    order = np.argsort(nk, kind="stable")
    return nk[order], nv[order], int((~present).sum())


def kv_delete(K, V, keys):
    """Removes the keys present; returns (K', V', number removed)."""
    gone = np.isin(K, _u64(keys))
    return K[~gone].copy(), V[~gone].copy(), int(gone.sum())


def kv_get(K, V, keys):
    q = _u64(keys)
    pos = np.searchsorted(K, q)
    ok = pos < len(K)
    found = np.zeros(len(q), dtype=np.uint8)
    found[ok] = (K[pos[ok]] == q[ok])
    val = np.zeros(len(q), dtype=np.uint64)
    val[found == 1] = V[pos[found == 1]]
    return val, found


def kv_range_values(K, V, lo, hi):
    """(sum of the values mod 2^64, count) of the keys in each [lo, hi)."""
    lo, hi = _u64(lo), _u64(hi)
    cs = np.concatenate([np.zeros(1, np.uint64), np.cumsum(V, dtype=np.uint64)])
    i0 = np.searchsorted(K, lo, side="left")
    i1 = np.searchsorted(K, hi, side="left")
    i1 = np.maximum(i0, i1)
    return cs[i1] - cs[i0], (i1 - i0).astype(np.uint64)


def decode_image(bytes_, used, S, cap):
    b = np.ascontiguousarray(bytes_, dtype=np.uint8)
    u = np.ascontiguousarray(used, dtype=np.uint32)
    out = np.empty(cap, dtype=np.uint64)
    m = lib().orc_decode_image(_p(b, ctypes.c_uint8), _p(u, ctypes.c_uint32), len(u), S,
                               _p(out, ctypes.c_uint64), cap)
    if m < 0:
        raise ValueError("malformed image")
    return out[:m].copy()


def bfs(edges, nv, src=0):
    e = _u64(edges)
    lv = np.empty(nv, dtype=np.uint32)
    lib().orc_bfs(_p(e, ctypes.c_uint64), len(e), nv, src, _p(lv, ctypes.c_uint32))
    return lv


def offsets(edges, nv):
    e = _u64(edges)
    off = np.empty(nv + 1, dtype=np.uint64)
    lib().orc_offsets(_p(e, ctypes.c_uint64), len(e), nv, _p(off, ctypes.c_uint64))
    return off


def cc(edges, nv):
    e = _u64(edges)
    lab = np.empty(nv, dtype=np.uint32)
    lib().orc_cc(_p(e, ctypes.c_uint64), len(e), nv, _p(lab, ctypes.c_uint32))
    return lab


def bc(edges, nv, src=0):
    """(sigma, delta) of Brandes' single-source betweenness from src."""
    e = _u64(edges)
    sg = np.empty(nv, dtype=np.float64)
    dl = np.empty(nv, dtype=np.float64)
    lib().orc_bc(_p(e, ctypes.c_uint64), len(e), nv, src, _p(sg, ctypes.c_double), _p(dl, ctypes.c_double))
    return sg, dl


def pagerank(edges, nv, iters=10, damping=0.85):
    e = _u64(edges)
    p = np.empty(nv, dtype=np.float64)
    lib().orc_pagerank(_p(e, ctypes.c_uint64), len(e), nv, iters, damping,
                       _p(p, ctypes.c_double))
    return p
