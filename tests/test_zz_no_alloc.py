"""The allocation-free bound sweep (sdfi_bounds_noalloc) against the entry
point with a caller workspace (sdfi_bounds): identical outputs on two calls
in a row, the second with a smaller input, in both precisions."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2605_01919_amd import sdfi
from sdfgen import configs

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def call(fn_name, samples, queries, precision):
    L = sdfi.lib()
    n, m = samples.shape[0], queries.shape[0]
    opt = sdfi.options(precision)
    out = [torch.full((m,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(2)]
    out += [torch.full((m,), -7, dtype=torch.int32, device="cuda") for _ in range(3)]
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in out]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if fn_name == "sdfi_bounds":
        ws = sdfi.workspace(sdfi.OP_BOUNDS, n, m, opt)
        st = L.sdfi_bounds(ctypes.c_void_p(samples.data_ptr()), ctypes.c_int64(n),
                           ctypes.c_void_p(queries.data_ptr()), ctypes.c_int64(m), *ptrs,
                           ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), ctypes.byref(opt), stream)
    else:
        st = L.sdfi_bounds_noalloc(ctypes.c_void_p(samples.data_ptr()), ctypes.c_int64(n),
                                   ctypes.c_void_p(queries.data_ptr()), ctypes.c_int64(m), *ptrs,
                                   ctypes.byref(opt), stream)
    assert st == 0, L.sdfi_last_error()
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_bounds_equal_workspace_bounds(precision):
    # the larger input first, then a smaller one: the scratch array keeps the
    # first call's contents, which must not leak into the second
    for w in (configs.ball_union(16, 1002), configs.sphere(6)):
        print("noalloc", precision, w.name, w.n, w.m, flush=True)
        s, q = dev(np.c_[w.points, w.values]), dev(w.queries)
        want = call("sdfi_bounds", s, q, precision)
        got = call("sdfi_bounds_noalloc", s, q, precision)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
