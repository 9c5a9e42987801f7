"""Thin Python binding of libsdfi.so (argument marshalling only).

Every function takes torch tensors that live on the GPU, passes their device
pointers and torch's current HIP stream to the C ABI declared in
include/sdfi.h, and returns torch tensors.  No computation happens here; if
the library is missing, the first call raises instead of computing anything
another way.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdfi.so")

PREC_FP64 = 0
PREC_FP32_FP64_RECHECK = 1

OP_BOUNDS, OP_CERTIFY, OP_ORDER, OP_WITNESS, OP_GREEDY, OP_RMIN, OP_REPAIR, OP_BACKWARD = range(8)

KIND_KEPT, KIND_HI, KIND_LO, KIND_ZERO, KIND_RMIN_T, KIND_RMIN_D, KIND_RMIN_U, KIND_COINCIDENT = range(8)
KIND_INFEASIBLE, KIND_UNRESOLVED = 254, 255

OPT_CERTIFY = 1
OPT_INPUT_CHECK = 2


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("tie_tol", ctypes.c_double), ("domain_lo", ctypes.c_double * 3),
                ("domain_hi", ctypes.c_double * 3), ("grid", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class Report(ctypes.Structure):
    _fields_ = [("pairs_evaluated", ctypes.c_int64), ("n_hi", ctypes.c_int64), ("n_lo", ctypes.c_int64),
                ("n_zero", ctypes.c_int64), ("n_rmin", ctypes.c_int64), ("n_coincident", ctypes.c_int64),
                ("n_infeasible", ctypes.c_int64), ("n_unresolved", ctypes.c_int64),
                ("n_fp64_rechecks", ctypes.c_int64), ("n_exact_searches", ctypes.c_int64),
                ("n_violations_pairwise", ctypes.c_int64), ("n_violations_witness", ctypes.c_int64),
                ("n_removed", ctypes.c_int64), ("ms_phase", ctypes.c_double * 8)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "ms_phase"}
        d["ms_phase"] = list(self.ms_phase)
        return d


class SdfiError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SdfiError(f"{LIB_PATH} is missing: build it with paper_2605_01919_amd/build.py "
                            "(or __graft_entry__.build()) before calling the GPU path")
        _lib = ctypes.CDLL(LIB_PATH)
        _lib.sdfi_last_error.restype = ctypes.c_char_p
        _lib.sdfi_version.restype = ctypes.c_char_p
        _lib.sdfi_default_options.argtypes = [ctypes.POINTER(Options)]
        _lib.sdfi_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]
    return _lib


EXPORTS = ["sdfi_default_options", "sdfi_last_error", "sdfi_version", "sdfi_workspace_size", "sdfi_bounds",
           "sdfi_certify", "sdfi_refinement_order", "sdfi_sample_witnesses", "sdfi_greedy_interpolate",
           "sdfi_greedy_interpolate_batched", "sdfi_min_valid_radius", "sdfi_repair", "sdfi_greedy_backward"]


def options(precision="fp32", grid=0, flags=0, tol=1e-6, tie_tol=1e-9, block_size=0):
    o = Options()
    lib().sdfi_default_options(ctypes.byref(o))
    o.precision = {"fp64": PREC_FP64, "fp32": PREC_FP32_FP64_RECHECK}[precision] if isinstance(precision, str) \
        else int(precision)
    o.grid = int(grid)
    o.flags = int(flags)
    o.tol = tol
    o.tie_tol = tie_tol
    o.block_size = block_size
    return o


def _check(status, what):
    if status != 0:
        msg = lib().sdfi_last_error().decode()
        raise SdfiError(f"{what} failed with status {status}: {msg}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape_last=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise SdfiError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise SdfiError(f"{name} must be {dtype}, got {t.dtype}")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise SdfiError(f"{name} must have shape (k, {shape_last}), got {tuple(t.shape)}")
    return t.contiguous()


def workspace(op, n, m, opt):
    size = ctypes.c_size_t()
    _check(lib().sdfi_workspace_size(op, n, m, ctypes.byref(opt), ctypes.byref(size)), "sdfi_workspace_size")
    return torch.empty(max(int(size.value), 256), dtype=torch.uint8, device="cuda")


def bounds(samples, queries, precision="fp32"):
    """lo, hi (float64), argmax, argmin (int32), flags (int32 bit pattern)."""
    samples = _dev(samples, torch.float64, 4, "samples")
    queries = _dev(queries, torch.float64, 3, "queries")
    n, m = samples.shape[0], queries.shape[0]
    opt = options(precision)
    dev = samples.device
    lo = torch.empty(m, dtype=torch.float64, device=dev)
    hi = torch.empty(m, dtype=torch.float64, device=dev)
    a = torch.empty(m, dtype=torch.int32, device=dev)
    b = torch.empty(m, dtype=torch.int32, device=dev)
    f = torch.empty(m, dtype=torch.int32, device=dev)
    ws = workspace(OP_BOUNDS, n, m, opt)
    _check(lib().sdfi_bounds(_ptr(samples), ctypes.c_int64(n), _ptr(queries), ctypes.c_int64(m), _ptr(lo),
                             _ptr(hi), _ptr(a), _ptr(b), _ptr(f), _ptr(ws), ctypes.c_size_t(ws.numel()),
                             ctypes.byref(opt), _stream()), "sdfi_bounds")
    return lo, hi, a, b, f


def certify(pts_values, witness):
    pts_values = _dev(pts_values, torch.float64, 4, "pts_values")
    witness = _dev(witness, torch.float64, 3, "witness")
    N = pts_values.shape[0]
    opt = options()
    rep = Report()
    ws = workspace(OP_CERTIFY, N, 0, opt)
    _check(lib().sdfi_certify(_ptr(pts_values), _ptr(witness), ctypes.c_int64(N), ctypes.byref(rep), _ptr(ws),
                              ctypes.c_size_t(ws.numel()), ctypes.byref(opt), _stream()), "sdfi_certify")
    return {"pair": rep.n_violations_pairwise, "witness": rep.n_violations_witness,
            "pairs_evaluated": rep.pairs_evaluated}
