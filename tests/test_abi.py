"""The C-ABI library loads and exports every entry point include/cpma.h declares
(no compute call: this container has no GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpma.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpma_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("cpma_build", "cpma_insert_batch", "cpma_delete_batch", "cpma_contains",
                 "cpma_range_map", "cpma_size", "cpma_bytes", "cpma_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2305_05055_amd as p
    if not os.path.exists(p.LIB_PATH):
        pytest.skip("libcpma.so not built")
    L = p.lib()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", p.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (cpma_[a-z_]+)$", out, flags=re.M))
    assert set(declared()) <= exported


def test_host_only_calls_without_gpu():
    """Calls that never touch the device behave as documented."""
    import ctypes
    import paper_2305_05055_amd as p
    if not os.path.exists(p.LIB_PATH):
        pytest.skip("libcpma.so not built")
    L = p.lib()
    c = p.default_config()
    assert c.leaf_bytes == 1024 and abs(c.grow - 1.2) < 1e-12
    assert abs(c.build_density - 0.7 / 1.2) < 1e-12
    assert L.cpma_size(None) == 0 and L.cpma_bytes(None) == 0
    assert L.cpma_config_default(None) == 1
    assert L.cpma_status_str(4) == b"reserved key (UINT64_MAX)"
    h = ctypes.c_void_p()
    assert L.cpma_build(None, 5, 0, None, None, ctypes.byref(h)) == 1   # keys NULL with n > 0
    bad = p.Config()
    bad.leaf_bytes = 100                                                 # not a power of two
    assert L.cpma_build(None, 0, 0, ctypes.byref(bad), None, ctypes.byref(h)) == 1
    assert L.cpma_insert_batch(None, None, 1, 0, 0, None, None) == 1
    assert L.cpma_range_map_noalloc(None, None, None, 1, None, None, None) == 1
    assert L.cpma_trim(None, None) == 1
    assert L.cpma_insert_kv(None, None, None, 1, 0, None, None) == 1
    assert L.cpma_get(None, None, 1, 0, None, None, None) == 1
    assert L.cpma_range_map_values(None, None, None, 1, 0, None, None, None) == 1
    assert L.cpma_export_code_bytes(None, None, None) == 1
    h = ctypes.c_void_p()
    kv_unc = p.Config()
    kv_unc.uncompressed = 1
    assert L.cpma_build_kv(None, None, 0, 0, ctypes.byref(kv_unc), None, ctypes.byref(h)) == 1
    assert L.cpma_stats_enable(None, 1) == 1
    assert L.cpma_stats_select(None, 1 << 2) == 1
    L.cpma_destroy(None)


def test_package_fails_loudly_without_library(monkeypatch):
    import paper_2305_05055_amd as p
    monkeypatch.setattr(p, "LIB_PATH", "/nonexistent/libcpma.so")
    monkeypatch.setattr(p, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        p.lib()


def test_package_does_not_import_oracle():
    src = open(os.path.join(ROOT, "paper_2305_05055_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
    for f in os.listdir(os.path.join(ROOT, "paper_2305_05055_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2305_05055_amd", "csrc", f)).read()


def test_server_argument_checks_without_gpu():
    import ctypes
    import paper_2305_05055_amd as p
    if not os.path.exists(p.LIB_PATH):
        pytest.skip("libcpma.so not built")
    L = p.lib()
    h = ctypes.c_void_p()
    assert L.cpma_server_start(None, None, ctypes.byref(h)) == 1
    assert L.cpma_server_submit(None, None) == 1
    assert L.cpma_server_stop(None, None) == 1
    t0 = p.clock_ns()
    assert p.clock_ns() >= t0 > 0
    assert ctypes.sizeof(p.Request) == 88


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of the C structs have the C compiler's sizes and offsets."""
    import ctypes
    import paper_2305_05055_amd as p
    prog = tmp_path / "sizes.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "cpma.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(cpma_config),"
        " offsetof(cpma_config, range_chunk), offsetof(cpma_config, alloc), offsetof(cpma_config, ctx),"
        " offsetof(cpma_config, rebuild_frac), offsetof(cpma_config, uncompressed),"
        " offsetof(cpma_config, values),"
        " sizeof(cpma_tune_hint), sizeof(cpma_tune_report),"
        " offsetof(cpma_tune_report, best_chunk), sizeof(cpma_request), sizeof(cpma_phase_stat));return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(p.Config), p.Config.range_chunk.offset, p.Config.alloc.offset, p.Config.ctx.offset,
            p.Config.rebuild_frac.offset, p.Config.uncompressed.offset, p.Config.values.offset,
            ctypes.sizeof(p.TuneHint),
            ctypes.sizeof(p.TuneReport), p.TuneReport.best_chunk.offset, ctypes.sizeof(p.Request),
            ctypes.sizeof(p.PhaseStat)]
    assert got == want


def test_config_defaults_and_checks_without_gpu():
    import ctypes
    import paper_2305_05055_amd as p
    if not os.path.exists(p.LIB_PATH):
        pytest.skip("libcpma.so not built")
    L = p.lib()
    c = p.default_config()
    assert c.range_chunk == 2
    h = ctypes.c_void_p()
    for S, chunk in ((8192, 0), (32, 0), (0, 3), (0, 128)):
        bad = p.Config()
        bad.leaf_bytes, bad.range_chunk = S, chunk
        assert L.cpma_build(None, 0, 0, ctypes.byref(bad), None, ctypes.byref(h)) == 1
    one_hook = p.Config()
    one_hook.alloc = 1  # an allocator without a matching free
    assert L.cpma_build(None, 0, 0, ctypes.byref(one_hook), None, ctypes.byref(h)) == 1
    out = p.Config()
    assert L.cpma_autotune(None, 0, 0, None, None, None, ctypes.byref(out), None) == 1
