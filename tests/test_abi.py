"""The C ABI library loads and exports every entry point of include/sdfi.h;
argument errors are caught on the host (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2605_01919_amd import sdfi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "sdfi.h")).read()
    return sorted(set(re.findall(r"\b(sdfi_[a-z_]+)\s*\(", text)))


def test_header_matches_binding_list():
    assert header_functions() == sorted(sdfi.EXPORTS)


def test_library_exports_every_symbol():
    out = subprocess.check_output(["nm", "-D", "--defined-only", sdfi.LIB_PATH]).decode()
    exported = set(re.findall(r" T (sdfi_\w+)", out))
    missing = [f for f in header_functions() if f not in exported]
    assert not missing, missing
    for f in header_functions():
        getattr(sdfi.lib(), f)


def test_defaults_and_version():
    o = sdfi.options()
    assert o.tol == 1e-6 and o.tie_tol == 1e-9 and o.struct_size == ctypes.sizeof(sdfi.Options)
    assert b"gfx950" in sdfi.lib().sdfi_version()


def test_argument_errors_on_host():
    L = sdfi.lib()
    o = sdfi.options()
    st = L.sdfi_bounds(None, ctypes.c_int64(10), None, ctypes.c_int64(5), None, None, None, None, None, None,
                       ctypes.c_size_t(0), ctypes.byref(o), None)
    assert st == 1 and b"null" in L.sdfi_last_error()
    st = L.sdfi_bounds(None, ctypes.c_int64(0), None, ctypes.c_int64(5), None, None, None, None, None, None,
                       ctypes.c_size_t(0), ctypes.byref(o), None)
    assert st == 1
    bad = sdfi.options()
    bad.struct_size = 3
    size = ctypes.c_size_t()
    assert L.sdfi_workspace_size(0, 10, 10, ctypes.byref(bad), ctypes.byref(size)) == 1
    bad = sdfi.options()
    bad.precision = 7
    assert L.sdfi_workspace_size(0, 10, 10, ctypes.byref(bad), ctypes.byref(size)) == 1
    rep = sdfi.Report()
    assert L.sdfi_certify(None, None, ctypes.c_int64(4), ctypes.byref(rep), None, ctypes.c_size_t(0),
                          ctypes.byref(o), None) == 1


def test_workspace_sizes_grow():
    o = sdfi.options()
    s1, s2 = ctypes.c_size_t(), ctypes.c_size_t()
    L = sdfi.lib()
    for op in range(8):
        assert L.sdfi_workspace_size(op, 100, 100, ctypes.byref(o), ctypes.byref(s1)) == 0
        assert L.sdfi_workspace_size(op, 10000, 10000, ctypes.byref(o), ctypes.byref(s2)) == 0
        assert s2.value >= s1.value > 0


def test_counters_and_block_size_on_host():
    L = sdfi.lib()
    v = ctypes.c_int64(-1)
    L.sdfi_timing_reset()
    assert L.sdfi_counter_query(b"sweep_pairs_skipped", ctypes.byref(v)) == 0 and v.value == 0
    assert L.sdfi_counter_query(b"no_such_counter", ctypes.byref(v)) == 0 and v.value == 0
    assert L.sdfi_counter_query(None, ctypes.byref(v)) == 1
    # 256 or 512 threads per greedy work-group (0 = 512); 4 wavefronts need
    # half the per-wavefront cap lists
    size = ctypes.c_size_t()
    sizes = {}
    for bs in (0, 256, 512):
        o = sdfi.options(block_size=bs)
        assert L.sdfi_workspace_size(4, 5000, 40000, ctypes.byref(o), ctypes.byref(size)) == 0
        sizes[bs] = size.value
    assert sizes[0] == sizes[512] > sizes[256]
    o = sdfi.options(block_size=1024)
    assert L.sdfi_workspace_size(4, 5000, 40000, ctypes.byref(o), ctypes.byref(size)) == 1
    assert b"block_size" in L.sdfi_last_error()
    # a batched launch adds a fixed amount per instance
    o = sdfi.options()
    assert L.sdfi_workspace_size(8, 0, 0, ctypes.byref(o), ctypes.byref(size)) == 0 and size.value > 0
    per_instance = size.value
    o = sdfi.options(groups=32)
    assert L.sdfi_workspace_size(8, 0, 0, ctypes.byref(o), ctypes.byref(size)) == 0 and size.value > per_instance
    o = sdfi.options(groups=-1)
    assert L.sdfi_workspace_size(8, 0, 0, ctypes.byref(o), ctypes.byref(size)) == 1
    assert b"groups" in L.sdfi_last_error()
    # the documented flags pass, any other bit is refused
    o = sdfi.options(flags=sdfi.OPT_CERTIFY | sdfi.OPT_INPUT_CHECK | sdfi.OPT_EXHAUSTIVE)
    assert L.sdfi_workspace_size(4, 5000, 40000, ctypes.byref(o), ctypes.byref(size)) == 0
    o = sdfi.options(flags=8)
    assert L.sdfi_workspace_size(4, 5000, 40000, ctypes.byref(o), ctypes.byref(size)) == 1
    assert b"flags" in L.sdfi_last_error()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    # rejected on the host before any device work (the dummy addresses are
    # never touched)
    L = sdfi.lib()
    o = sdfi.options()
    fake = [ctypes.c_void_p(256 * (k + 1)) for k in range(7)]
    st = L.sdfi_bounds_noalloc(fake[0], ctypes.c_int64(262144), fake[1], ctypes.c_int64(2097152), *fake[2:],
                               ctypes.byref(o), None)
    assert st == 6 and b"scratch" in L.sdfi_last_error()
    st = L.sdfi_bounds_noalloc(None, ctypes.c_int64(10), None, ctypes.c_int64(5), None, None, None, None, None,
                               ctypes.byref(o), None)
    assert st == 1
