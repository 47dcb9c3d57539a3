"""Python binding of the MI355X CPMA (C ABI in include/cpma.h).

Argument marshalling only: every step of build / insert_batch / delete_batch /
contains / range_map runs in the HIP kernels of libcpma.so.  Host inputs are
numpy arrays (uint64); device inputs are torch tensors on the GPU (int64 or
uint64 storage, the bit pattern is the key), passed with the current torch
stream.  There is no CPU fallback: without the built library every call raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpma.so")

MEM_HOST = 0
MEM_DEVICE = 1
NOALLOC_MAX_QUERIES = 65536  # CPMA_NOALLOC_MAX_QUERIES

STATUS = {0: "ok", 1: "invalid argument", 2: "device allocation failed", 3: "device error",
          4: "reserved key (UINT64_MAX)"}


class CpmaError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("leaf_bytes", ctypes.c_uint32), ("grow", ctypes.c_double),
                ("up_leaf", ctypes.c_double), ("up_root", ctypes.c_double),
                ("lo_leaf", ctypes.c_double), ("lo_root", ctypes.c_double),
                ("build_density", ctypes.c_double), ("range_chunk", ctypes.c_uint32),
                ("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p), ("ctx", ctypes.c_void_p),
                ("rebuild_frac", ctypes.c_double), ("uncompressed", ctypes.c_int32),
                ("values", ctypes.c_int32)]


class TuneHint(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_uint64), ("range_keys", ctypes.c_uint64), ("queries", ctypes.c_uint64),
                ("sample_keys", ctypes.c_uint64), ("insert_weight", ctypes.c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("sample_n", ctypes.c_uint64), ("leaf_bytes", ctypes.c_uint32 * 5),
                ("insert_ms", ctypes.c_double * 5), ("range_ms", ctypes.c_double * 5),
                ("chunk", ctypes.c_uint32 * 6), ("chunk_ms", ctypes.c_double * 6),
                ("best_leaf_bytes", ctypes.c_uint32), ("best_chunk", ctypes.c_uint32),
                ("rebuild_ms", ctypes.c_double), ("batch_path_ms", ctypes.c_double),
                ("best_rebuild_frac", ctypes.c_double)]


class Request(ctypes.Structure):
    """cpma_request: one range batch, insert batch or delete batch for the server."""
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("keys", ctypes.c_void_p), ("hi", ctypes.c_void_p), ("sum", ctypes.c_void_p),
                ("count", ctypes.c_void_p), ("result", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("done", ctypes.c_int32), ("t_done_ns", ctypes.c_uint64), ("step", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_slots", ctypes.c_uint32)]


REQ_RANGE, REQ_INSERT, REQ_DELETE = 0, 1, 2


class PhaseStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("ms", ctypes.c_double), ("alg_bytes", ctypes.c_uint64)]


PHASES = ("sort", "locate", "merge", "heavy", "count", "redist", "range_scan", "query")

_lib = None


def lib():
    """Loads libcpma.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcpma.so is not built: run __graft_entry__.build() "
                               "(or python -m paper_2305_05055_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        u64 = ctypes.c_uint64
        L.cpma_config_default.argtypes = [ctypes.POINTER(Config)]
        L.cpma_build.argtypes = [vp, u64, ctypes.c_int, ctypes.POINTER(Config), vp,
                                 ctypes.POINTER(vp)]
        L.cpma_insert_batch.argtypes = [vp, vp, u64, ctypes.c_int, ctypes.c_int, vp,
                                        ctypes.POINTER(u64)]
        L.cpma_delete_batch.argtypes = L.cpma_insert_batch.argtypes
        L.cpma_apply_updates.argtypes = [vp, ctypes.c_uint32, vp, vp, vp, ctypes.c_int, vp, vp]
        L.cpma_contains.argtypes = [vp, vp, u64, ctypes.c_int, vp, vp]
        L.cpma_range_map.argtypes = [vp, vp, vp, u64, ctypes.c_int, vp, vp, vp]
        L.cpma_range_map_noalloc.argtypes = [vp, vp, vp, u64, vp, vp, vp]
        L.cpma_size.argtypes = [vp]
        L.cpma_size.restype = u64
        L.cpma_bytes.argtypes = [vp]
        L.cpma_bytes.restype = u64
        L.cpma_bytes_held.argtypes = [vp]
        L.cpma_bytes_held.restype = u64
        L.cpma_trim.argtypes = [vp, vp]
        L.cpma_build_kv.argtypes = [vp, vp, u64, ctypes.c_int, vp, vp, ctypes.POINTER(vp)]
        L.cpma_insert_kv.argtypes = [vp, vp, vp, u64, ctypes.c_int, vp, ctypes.POINTER(u64)]
        L.cpma_get.argtypes = [vp, vp, u64, ctypes.c_int, vp, vp, vp]
        L.cpma_range_map_values.argtypes = [vp, vp, vp, u64, ctypes.c_int, vp, vp, vp]
        L.cpma_export_code_bytes.argtypes = [vp, vp, vp]
        L.cpma_geometry.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_uint32)]
        L.cpma_export.argtypes = [vp, vp, vp, vp, vp]
        L.cpma_destroy.argtypes = [vp]
        L.cpma_destroy.restype = None
        L.cpma_fgraph_bfs.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, vp, vp]
        L.cpma_fgraph_offsets.argtypes = [vp, ctypes.c_uint32, ctypes.c_int, vp, vp]
        L.cpma_fgraph_cc.argtypes = [vp, ctypes.c_uint32, ctypes.c_int, vp, vp]
        L.cpma_fgraph_bc.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, vp, vp, vp]
        L.cpma_fgraph_pagerank.argtypes = [vp, ctypes.c_uint32, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int, vp, vp]
        L.cpma_server_start.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
        L.cpma_server_submit.argtypes = [vp, ctypes.POINTER(Request)]
        L.cpma_server_stop.argtypes = [vp, ctypes.POINTER(u64)]
        L.cpma_clock_ns.argtypes = []
        L.cpma_clock_ns.restype = u64
        L.cpma_stats_enable.argtypes = [vp, ctypes.c_int]
        L.cpma_stats_select.argtypes = [vp, ctypes.c_uint32]
        L.cpma_stats_get.argtypes = [vp, ctypes.POINTER(PhaseStat), ctypes.c_int]
        L.cpma_autotune.argtypes = [vp, u64, ctypes.c_int, ctypes.POINTER(TuneHint), ctypes.POINTER(Config),
                                    vp, ctypes.POINTER(Config), ctypes.POINTER(TuneReport)]
        L.cpma_status_str.argtypes = [ctypes.c_int]
        L.cpma_status_str.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code, what):
    if code != 0:
        raise CpmaError(code, what)


def _is_torch_cuda(x):
    return hasattr(x, "is_cuda") and x.is_cuda


def _stream(stream, device_args):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    if device_args:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


def _keys(x):
    """(pointer, length, memspace, keepalive) for a key array."""
    if _is_torch_cuda(x):
        import torch
        if x.dtype not in (torch.int64, torch.uint64):
            raise TypeError("device keys must be int64/uint64 tensors")
        x = x.contiguous()
        return ctypes.c_void_p(x.data_ptr()), x.numel(), MEM_DEVICE, x
    a = np.ascontiguousarray(x, dtype=np.uint64)
    return ctypes.c_void_p(a.ctypes.data), len(a), MEM_HOST, a


def default_config():
    c = Config()
    lib().cpma_config_default(ctypes.byref(c))
    return c


def autotune(keys, batch=0, range_keys=0, queries=0, sample_keys=0, insert_weight=-1.0, base=None,
             stream=None):
    """cpma_autotune: (Config with the chosen leaf_bytes, range_chunk and rebuild_frac, report dict)."""
    p, n, mem, keep = _keys(keys)
    hint = TuneHint(batch, range_keys, queries, sample_keys, insert_weight)
    out = Config()
    rep = TuneReport()
    _check(lib().cpma_autotune(p if n else None, n, mem, ctypes.byref(hint),
                               ctypes.byref(base) if base is not None else None,
                               _stream(stream, mem == MEM_DEVICE), ctypes.byref(out), ctypes.byref(rep)),
           "cpma_autotune")
    report = {"sample_n": rep.sample_n, "best_leaf_bytes": rep.best_leaf_bytes, "best_chunk": rep.best_chunk,
              "leaf_bytes": {int(rep.leaf_bytes[i]): {"insert_ms": rep.insert_ms[i], "range_ms": rep.range_ms[i]}
                             for i in range(5)},
              "range_chunk_ms": {int(rep.chunk[i]): rep.chunk_ms[i] for i in range(6)},
              "rebuild_ms": rep.rebuild_ms, "batch_path_ms": rep.batch_path_ms,
              "best_rebuild_frac": rep.best_rebuild_frac}
    return out, report


class CPMA:
    """A device-resident compressed packed memory array of uint64 keys."""

    def __init__(self, keys=(), leaf_bytes=0, grow=0.0, bounds=None, build_density=0.0,
                 stream=None, config=None, range_chunk=0, uncompressed=False, values=None):
        """uncompressed=True builds the plain PMA (raw 8-byte keys per leaf);
        values (an array beside keys, same memory space) builds a key-value set."""
        if config is not None:
            cfg = Config.from_buffer_copy(config)
        else:
            cfg = Config()
            cfg.leaf_bytes = leaf_bytes
            cfg.grow = grow
            if bounds is not None:
                cfg.up_leaf, cfg.up_root, cfg.lo_leaf, cfg.lo_root = bounds
            cfg.build_density = build_density
            cfg.range_chunk = range_chunk
            cfg.uncompressed = 1 if uncompressed else 0
        p, n, mem, keep = _keys(keys)
        h = ctypes.c_void_p()
        if values is not None:
            pv, nv, memv, keepv = _keys(values)
            if nv != n or memv != mem:
                raise ValueError("values must match keys in length and memory space")
            _check(lib().cpma_build_kv(p if n else None, pv if n else None, n, mem, ctypes.byref(cfg),
                                       _stream(stream, mem == MEM_DEVICE), ctypes.byref(h)), "cpma_build_kv")
            keep = (keep, keepv)
        else:
            _check(lib().cpma_build(p if n else None, n, mem, ctypes.byref(cfg),
                                    _stream(stream, mem == MEM_DEVICE), ctypes.byref(h)), "cpma_build")
        self._h = h
        self._keep = keep

    def close(self):
        if getattr(self, "_h", None):
            lib().cpma_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _update(self, fn, keys, sorted, stream, what):
        p, k, mem, keep = _keys(keys)
        out = ctypes.c_uint64(0)
        _check(fn(self._h, p if k else None, k, mem, 1 if sorted else 0,
                  _stream(stream, mem == MEM_DEVICE), ctypes.byref(out)), what)
        return int(out.value)

    def insert_batch(self, keys, sorted=False, stream=None):
        """Inserts keys; returns how many were not present before."""
        return self._update(lib().cpma_insert_batch, keys, sorted, stream, "cpma_insert_batch")

    def insert_kv(self, keys, values, stream=None):
        """Inserts or overwrites key-value pairs; returns how many keys were new."""
        p, k, mem, keep = _keys(keys)
        pv, kv, memv, keepv = _keys(values)
        if kv != k or memv != mem:
            raise ValueError("values must match keys in length and memory space")
        out = ctypes.c_uint64(0)
        _check(lib().cpma_insert_kv(self._h, p if k else None, pv if k else None, k, mem,
                                    _stream(stream, mem == MEM_DEVICE), ctypes.byref(out)), "cpma_insert_kv")
        return int(out.value)

    def get(self, keys, stream=None):
        """(values, found) of a key-value set for each key."""
        p, q, mem, keep = _keys(keys)
        if mem == MEM_DEVICE:
            import torch
            v = torch.empty(q, dtype=torch.int64, device=keys.device)
            f = torch.empty(q, dtype=torch.uint8, device=keys.device)
            pv, pf = ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(f.data_ptr())
        else:
            v = np.empty(q, dtype=np.uint64)
            f = np.empty(q, dtype=np.uint8)
            pv, pf = ctypes.c_void_p(v.ctypes.data), ctypes.c_void_p(f.ctypes.data)
        _check(lib().cpma_get(self._h, p, q, mem, pv, pf, _stream(stream, mem == MEM_DEVICE)), "cpma_get")
        return v, f

    def range_map_values(self, lo, hi, stream=None):
        """(sum of the values mod 2^64, count) of the keys in each [lo[i], hi[i])."""
        return self.range_map(lo, hi, stream, _fn=lib().cpma_range_map_values, _what="cpma_range_map_values")

    def code_bytes(self, stream=None):
        """Each leaf's key code bytes (key-value sets)."""
        L, _ = self.geometry()
        c = np.empty(L, dtype=np.uint32)
        _check(lib().cpma_export_code_bytes(self._h, ctypes.c_void_p(c.ctypes.data), _stream(stream, False)),
               "cpma_export_code_bytes")
        return c

    def delete_batch(self, keys, sorted=False, stream=None):
        """Deletes keys; returns how many were present."""
        return self._update(lib().cpma_delete_batch, keys, sorted, stream, "cpma_delete_batch")

    def apply_updates(self, requests, stream=None):
        """Applies [(kind, keys), ...] (kind REQ_INSERT or REQ_DELETE; keys host
        arrays or device tensors, all in one memory space) as if one
        insert_batch / delete_batch call ran per request in order, with one
        fused pass; returns each request's count."""
        nreq = len(requests)
        kinds = np.array([int(k) for k, _ in requests], dtype=np.int32)
        ptrs = np.zeros(nreq, dtype=np.uint64)
        ns = np.zeros(nreq, dtype=np.uint64)
        keep, mem = [], MEM_HOST
        for i, (_, ks) in enumerate(requests):
            p, k, m, kp = _keys(ks)
            if i == 0:
                mem = m
            elif m != mem:
                raise ValueError("all requests' keys must be in one memory space")
            keep.append(kp)
            ptrs[i] = p.value if (k and p is not None and p.value) else 0
            ns[i] = k
        res = np.zeros(nreq, dtype=np.uint64)
        _check(lib().cpma_apply_updates(self._h, nreq, ctypes.c_void_p(kinds.ctypes.data),
                                        ctypes.c_void_p(ptrs.ctypes.data), ctypes.c_void_p(ns.ctypes.data),
                                        mem, ctypes.c_void_p(res.ctypes.data),
                                        _stream(stream, mem == MEM_DEVICE)), "cpma_apply_updates")
        return [int(x) for x in res]

    def contains(self, keys, stream=None):
        p, q, mem, keep = _keys(keys)
        if mem == MEM_DEVICE:
            import torch
            out = torch.empty(q, dtype=torch.uint8, device=keys.device)
            optr = ctypes.c_void_p(out.data_ptr())
        else:
            out = np.empty(q, dtype=np.uint8)
            optr = ctypes.c_void_p(out.ctypes.data)
        _check(lib().cpma_contains(self._h, p, q, mem, optr, _stream(stream, mem == MEM_DEVICE)),
               "cpma_contains")
        return out

    def range_map(self, lo, hi, stream=None, _fn=None, _what="cpma_range_map"):
        """(sum mod 2^64, count) of the keys in each [lo[i], hi[i])."""
        plo, q, mem, klo = _keys(lo)
        phi, q2, mem2, khi = _keys(hi)
        if q != q2 or mem != mem2:
            raise ValueError("lo and hi must have the same length and memory space")
        if mem == MEM_DEVICE:
            import torch
            s = torch.empty(q, dtype=torch.int64, device=lo.device)
            c = torch.empty(q, dtype=torch.int64, device=lo.device)
            ps, pc = ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(c.data_ptr())
        else:
            s = np.empty(q, dtype=np.uint64)
            c = np.empty(q, dtype=np.uint64)
            ps, pc = ctypes.c_void_p(s.ctypes.data), ctypes.c_void_p(c.ctypes.data)
        _check((_fn or lib().cpma_range_map)(self._h, plo, phi, q, mem, ps, pc,
                                             _stream(stream, mem == MEM_DEVICE)), _what)
        return s, c

    def range_map_noalloc(self, lo, hi, sum_out=None, count_out=None, stream=None):
        """range_map through the entry point that allocates nothing: lo, hi and
        the outputs are device tensors (outputs allocated here by torch unless
        given), at most NOALLOC_MAX_QUERIES queries."""
        plo, q, mem, klo = _keys(lo)
        phi, q2, mem2, khi = _keys(hi)
        if q != q2 or mem != MEM_DEVICE or mem2 != MEM_DEVICE:
            raise ValueError("lo and hi must be device tensors of the same length")
        import torch
        s = torch.empty(q, dtype=torch.int64, device=lo.device) if sum_out is None else sum_out
        c = torch.empty(q, dtype=torch.int64, device=lo.device) if count_out is None else count_out
        _check(lib().cpma_range_map_noalloc(self._h, plo, phi, q, ctypes.c_void_p(s.data_ptr()),
                                            ctypes.c_void_p(c.data_ptr()), _stream(stream, True)),
               "cpma_range_map_noalloc")
        return s, c

    def __len__(self):
        return int(lib().cpma_size(self._h))

    def size(self):
        return int(lib().cpma_size(self._h))

    def bytes(self):
        return int(lib().cpma_bytes(self._h))

    def bytes_held(self):
        """All device bytes the handle holds (structure, spare arrays, scratch)."""
        return int(lib().cpma_bytes_held(self._h))

    def trim(self, stream=None):
        """Releases the spare arrays and every scratch buffer kept from earlier calls."""
        _check(lib().cpma_trim(self._h, _stream(stream, True)), "cpma_trim")

    def geometry(self):
        L = ctypes.c_uint64(0)
        S = ctypes.c_uint32(0)
        _check(lib().cpma_geometry(self._h, ctypes.byref(L), ctypes.byref(S)), "cpma_geometry")
        return int(L.value), int(S.value)

    # ---- F-Graph: edge keys u<<32 | v --------------------------------------------
    def bfs(self, nv, source=0, symmetric=False, device=False, stream=None):
        """Hop distance of every vertex from `source` (0xFFFFFFFF if unreachable).
        symmetric=True promises every edge has its reverse (allows bottom-up levels)."""
        if device:
            import torch
            out = torch.empty(nv, dtype=torch.int32, device="cuda")
            ptr, mem = ctypes.c_void_p(out.data_ptr()), MEM_DEVICE
        else:
            out = np.empty(nv, dtype=np.uint32)
            ptr, mem = ctypes.c_void_p(out.ctypes.data), MEM_HOST
        _check(lib().cpma_fgraph_bfs(self._h, nv, source, 1 if symmetric else 0, mem, ptr,
                                     _stream(stream, device)),
               "cpma_fgraph_bfs")
        return out

    def pagerank(self, nv, iters=10, damping=0.85, device=False, stream=None):
        """FP32 PageRank after `iters` rounds from the uniform vector."""
        if device:
            import torch
            out = torch.empty(nv, dtype=torch.float32, device="cuda")
            ptr, mem = ctypes.c_void_p(out.data_ptr()), MEM_DEVICE
        else:
            out = np.empty(nv, dtype=np.float32)
            ptr, mem = ctypes.c_void_p(out.ctypes.data), MEM_HOST
        _check(lib().cpma_fgraph_pagerank(self._h, nv, iters, damping, mem, ptr,
                                          _stream(stream, device)), "cpma_fgraph_pagerank")
        return out

    def _out(self, n, np_dtype, torch_dtype, device):
        if device:
            import torch
            out = torch.empty(n, dtype=torch_dtype, device="cuda")
            return out, ctypes.c_void_p(out.data_ptr()), MEM_DEVICE
        out = np.empty(n, dtype=np_dtype)
        return out, ctypes.c_void_p(out.ctypes.data), MEM_HOST

    def offsets(self, nv, device=False, stream=None):
        """Vertex offset array: off[v] = number of edges with source below v (nv + 1 entries)."""
        import torch
        out, ptr, mem = self._out(nv + 1, np.uint64, torch.int64, device)
        _check(lib().cpma_fgraph_offsets(self._h, nv, mem, ptr, _stream(stream, device)), "cpma_fgraph_offsets")
        return out

    def cc(self, nv, device=False, stream=None):
        """Connected components: the smallest vertex id of each vertex's component."""
        import torch
        out, ptr, mem = self._out(nv, np.uint32, torch.int32, device)
        _check(lib().cpma_fgraph_cc(self._h, nv, mem, ptr, _stream(stream, device)), "cpma_fgraph_cc")
        return out

    def bc(self, nv, source=0, device=False, stream=None):
        """Single-source betweenness from `source`: (sigma, delta), FP64."""
        import torch
        sg, psg, mem = self._out(nv, np.float64, torch.float64, device)
        dl, pdl, _ = self._out(nv, np.float64, torch.float64, device)
        _check(lib().cpma_fgraph_bc(self._h, nv, source, mem, psg, pdl, _stream(stream, device)), "cpma_fgraph_bc")
        return sg, dl

    def stats_enable(self, on=True):
        """Starts (zeroing) or stops per-phase HIP-event timing inside the library."""
        _check(lib().cpma_stats_enable(self._h, 1 if on else 0), "cpma_stats_enable")

    def stats_select(self, phases):
        """Starts (zeroing) HIP-event timing of the named phases only (see PHASES);
        an empty list stops it."""
        mask = 0
        for name in phases:
            mask |= 1 << PHASES.index(name)
        _check(lib().cpma_stats_select(self._h, mask), "cpma_stats_select")

    def stats(self):
        """{phase: (launches, ms, algorithmic bytes)} accumulated since stats_enable."""
        arr = (PhaseStat * len(PHASES))()
        _check(lib().cpma_stats_get(self._h, arr, len(PHASES)), "cpma_stats_get")
        return {name: (int(arr[i].launches), float(arr[i].ms), int(arr[i].alg_bytes))
                for i, name in enumerate(PHASES)}

    def export(self, stream=None):
        """Host copies (bytes[L*S] u8, used[L] u32, head[L] u64) of the layout."""
        L, S = self.geometry()
        b = np.empty(L * S, dtype=np.uint8)
        u = np.empty(L, dtype=np.uint32)
        h = np.empty(L, dtype=np.uint64)
        _check(lib().cpma_export(self._h, ctypes.c_void_p(b.ctypes.data), ctypes.c_void_p(u.ctypes.data),
                                 ctypes.c_void_p(h.ctypes.data), _stream(stream, False)), "cpma_export")
        return b, u, h


def clock_ns():
    """Steady-clock nanoseconds (the clock of a request's t_done_ns)."""
    return int(lib().cpma_clock_ns())


class ServedRequest:
    """A request plus the host arrays it points to (kept alive until done)."""

    def __init__(self, kind, keys, hi=None):
        self.kind = kind
        self.keys = np.ascontiguousarray(keys, dtype=np.uint64)
        self.hi = None if hi is None else np.ascontiguousarray(hi, dtype=np.uint64)
        n = len(self.keys)
        self.sum = np.zeros(n, dtype=np.uint64) if kind == REQ_RANGE else None
        self.count = np.zeros(n, dtype=np.uint64) if kind == REQ_RANGE else None
        self.req = Request()
        self.req.kind = kind
        self.req.n = n
        self.req.keys = self.keys.ctypes.data if n else None
        self.req.hi = self.hi.ctypes.data if self.hi is not None and n else None
        self.req.sum = self.sum.ctypes.data if self.sum is not None and n else None
        self.req.count = self.count.ctypes.data if self.count is not None and n else None
        self.t_submit_ns = 0

    @property
    def done(self):
        return self.req.done != 0


class Server:
    """Serving loop over one CPMA (native worker thread; see cpma_server_* in cpma.h)."""

    def __init__(self, cpma_obj, hbm_budget=0, max_slots=0):
        cfg = ServerConfig(hbm_budget, max_slots)
        h = ctypes.c_void_p()
        _check(lib().cpma_server_start(cpma_obj.handle, ctypes.byref(cfg), ctypes.byref(h)),
               "cpma_server_start")
        self._h = h
        self._set = cpma_obj

    def submit(self, sr):
        sr.t_submit_ns = clock_ns()
        _check(lib().cpma_server_submit(self._h, ctypes.byref(sr.req)), "cpma_server_submit")

    def stop(self):
        steps = ctypes.c_uint64(0)
        if self._h:
            _check(lib().cpma_server_stop(self._h, ctypes.byref(steps)), "cpma_server_stop")
            self._h = None
        return int(steps.value)
