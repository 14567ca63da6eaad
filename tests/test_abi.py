"""CPU checks of the C-ABI library: it loads, exports every function that
include/*.h declares, and rejects bad arguments on the host before any GPU
call.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

from paper_2504_18211_amd import hbheap as hb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h") or fn == "hbheap_device.h":
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\([^;{]*\)\s*;", text, re.M):
            if m.group(1) not in ("if", "while", "for", "return"):
                names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hb.LIB_PATH):
        from paper_2504_18211_amd import build
        build.build()
    return hb.lib()


def test_exports_every_declared_symbol(L):
    declared = _declared_functions()
    assert {"heap_create", "heap_destroy", "heap_alloc_batch", "heap_free_batch"} <= declared
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} declared in include/ but not exported"
    assert set(hb.EXPORTS) <= declared


def test_version(L):
    assert "gfx950" in hb.hbheap_version()


@pytest.mark.parametrize("nbytes,chunk", [(1 << 20, 3000), (1 << 20, 2048), (1 << 20, 1 << 17), (4096, 8192)])
def test_create_rejects_bad_geometry(L, nbytes, chunk):
    out = C.c_void_p(0)
    assert L.heap_create(nbytes, chunk, C.byref(out)) == hb.E_INVAL
    assert out.value is None


def test_create_rejects_bad_config(L):
    out = C.c_void_p(0)
    for cfg in [hb.HeapConfig(6, 64, 0, 0, 0), hb.HeapConfig(0, 48, 0, 0, 0), hb.HeapConfig(0, 128, 0, 0, 0)]:
        assert L.heap_create_ex(1 << 20, 8192, C.byref(cfg), C.byref(out)) == hb.E_INVAL
    # page variant data region above 64 GiB
    assert L.heap_create_ex(65 << 30, 8192, C.byref(hb.HeapConfig(1, 64, 0, 0, 0)), C.byref(out)) == hb.E_INVAL
    assert L.heap_create(1 << 20, 8192, None) == hb.E_INVAL


def test_null_handle_and_buffers_rejected(L):
    assert L.heap_alloc_batch(None, None, None, 5, None) == hb.E_INVAL
    assert L.heap_free_batch(None, None, None, 5, None) == hb.E_INVAL
    assert L.heap_trim(None, None) == hb.E_INVAL
    assert L.heap_destroy(None) == hb.OK
    assert L.heap_replay(None, None, None, 1, None) == hb.E_INVAL
    assert L.heap_pattern_write(None, None, None, 3, 0, None) == hb.E_INVAL
    assert L.hb_atomic_probe(9, None, 0, 1, 1, 1, None) == hb.E_INVAL
    assert L.hb_stream_copy(None, None, 16, None) == hb.E_INVAL
    d = hb.DevHandle()
    assert L.heap_device_handle(None, C.byref(d)) == hb.E_INVAL


def test_dev_handle_layout_matches_header():
    # 11 pointers, one u64, twelve u32; virtualised array: 4 pointers, four u32, one u64;
    # eager retirement: one pointer
    assert C.sizeof(hb.DevHandle) == 11 * 8 + 8 + 12 * 4 + 4 * 8 + 4 * 4 + 8 + 8


def test_growth_rejects_bad_arguments(L):
    out = C.c_void_p(0)
    assert L.growth_create(None, 10, None, 9, 0, C.byref(out)) == hb.E_INVAL
    assert out.value is None
    assert L.growth_destroy(None) == hb.OK
    assert L.growth_step(None, 0, None) == hb.E_INVAL
    assert L.growth_graph_launch(None, None) == hb.E_INVAL
    assert L.growth_release(None, None) == hb.E_INVAL
    assert L.growth_export(None, None, None, None, None) == hb.E_INVAL
    b, t = C.c_uint32(), C.c_uint32()
    assert L.growth_launch_shape(None, C.byref(b), C.byref(t)) == hb.E_INVAL
    ms = (C.c_float * 1)()
    best = C.c_int32()
    assert L.growth_autotune(1 << 20, 10, None, 9, 0, None, 0, 1, ms, C.byref(best)) == hb.E_INVAL


def test_serve_rejects_bad_arguments(L):
    out = C.c_void_p(0)
    cfg = hb.ServeConfig(4, 4096, 1000, 0.95, 1, 1)
    assert L.serve_create(None, C.byref(cfg), C.byref(out)) == hb.E_INVAL
    assert out.value is None
    assert L.serve_destroy(None) == hb.OK
    st = hb.ServeStats()
    assert L.serve_run(None, 0, None, None, None, 1, None, None, None, None, None, C.byref(st)) == hb.E_INVAL
    assert L.serve_export(None, 0, 1, None, None) == hb.E_INVAL
    v = C.c_uint64()
    assert L.heap_chunks_in_use(None, C.byref(v), None) == hb.E_INVAL


def test_normal_build_has_no_fuzz_points(L):
    """Schedule fuzzing exists only in the test build (libhbheap_fuzz.so):
    the normal library refuses it, with no GPU call."""
    assert L.hb_fuzz_set(1, 8) == hb.E_UNSUP


def test_fuzz_build_exports_the_allocator():
    """The test build carries the allocator's entry points and the setter."""
    import os
    if not os.path.exists(hb.FUZZ_LIB_PATH):
        pytest.fail(f"{hb.FUZZ_LIB_PATH} is missing: build it with __graft_entry__.build()")
    F = C.CDLL(hb.FUZZ_LIB_PATH)
    for name in ("heap_create_ex", "heap_alloc_batch", "heap_free_batch", "heap_trim", "heap_snapshot",
                 "heap_pattern_write", "heap_pattern_check", "hb_fuzz_set"):
        assert hasattr(F, name), name


def test_host_malloc_sweep_runs_on_the_host(L):
    """The host malloc/free context figure needs no GPU: rounds are timed,
    nothing fails, and bad arguments are refused."""
    secs, failed = hb.hb_host_malloc_sweep([16, 4096], 1 << 12, 2, 2)
    assert secs.shape == (2, 2) and (secs > 0).all() and failed == 0
    out = (C.c_double * 2)()
    f = C.c_uint64()
    sizes = (C.c_uint64 * 1)(16)
    assert L.hb_host_malloc_sweep(sizes, 1, 16, 2, 0, out, C.byref(f)) == hb.E_INVAL   # no threads
    assert L.hb_host_malloc_sweep(None, 1, 16, 2, 1, out, C.byref(f)) == hb.E_INVAL
    assert L.hb_host_malloc_sweep(sizes, 1, 16, 0, 1, out, C.byref(f)) == hb.E_INVAL  # no rounds
