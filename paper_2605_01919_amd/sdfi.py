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

OP_BOUNDS, OP_CERTIFY, OP_ORDER, OP_WITNESS, OP_GREEDY, OP_RMIN, OP_REPAIR, OP_BACKWARD, OP_GREEDY_INSTANCE = range(9)

KIND_KEPT, KIND_HI, KIND_LO, KIND_ZERO, KIND_RMIN_T, KIND_RMIN_D, KIND_RMIN_U, KIND_COINCIDENT = range(8)
KIND_INFEASIBLE, KIND_UNRESOLVED = 254, 255

OPT_CERTIFY = 1
OPT_INPUT_CHECK = 2
OPT_EXHAUSTIVE = 4


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("tie_tol", ctypes.c_double), ("domain_lo", ctypes.c_double * 3),
                ("domain_hi", ctypes.c_double * 3), ("grid", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("groups", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("pairs_evaluated", ctypes.c_int64), ("n_hi", ctypes.c_int64), ("n_lo", ctypes.c_int64),
                ("n_zero", ctypes.c_int64), ("n_rmin", ctypes.c_int64), ("n_coincident", ctypes.c_int64),
                ("n_infeasible", ctypes.c_int64), ("n_unresolved", ctypes.c_int64),
                ("n_fp64_rechecks", ctypes.c_int64), ("n_exact_searches", ctypes.c_int64),
                ("n_violations_pairwise", ctypes.c_int64), ("n_violations_witness", ctypes.c_int64),
                ("n_removed", ctypes.c_int64), ("n_search_capped", ctypes.c_int64),
                ("ms_phase", ctypes.c_double * 8)]

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


EXPORTS = ["sdfi_default_options", "sdfi_last_error", "sdfi_version", "sdfi_timing_enable", "sdfi_timing_query",
           "sdfi_counter_query", "sdfi_timing_reset", "sdfi_workspace_size", "sdfi_bounds", "sdfi_bounds_noalloc",
           "sdfi_certify", "sdfi_refinement_order", "sdfi_sample_witnesses", "sdfi_greedy_interpolate",
           "sdfi_greedy_interpolate_batched", "sdfi_min_valid_radius", "sdfi_repair", "sdfi_greedy_backward"]


def options(precision="fp32", grid=0, flags=0, tol=1e-6, tie_tol=1e-9, block_size=0, groups=0):
    o = Options()
    lib().sdfi_default_options(ctypes.byref(o))
    o.precision = {"fp64": PREC_FP64, "fp32": PREC_FP32_FP64_RECHECK}[precision] if isinstance(precision, str) \
        else int(precision)
    o.grid = int(grid)
    o.flags = int(flags)
    o.tol = tol
    o.tie_tol = tie_tol
    o.block_size = block_size
    o.groups = int(groups)
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
    if shape_last is None and t.dim() != 1:
        raise SdfiError(f"{name} must be one-dimensional, got {tuple(t.shape)}")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise SdfiError(f"{name} must have shape (k, {shape_last}), got {tuple(t.shape)}")
    return t.contiguous()


def timing(on=True):
    """Enable or disable the library's kernel timing (HIP events on the caller's stream)."""
    if on:
        lib().sdfi_timing_reset()
    lib().sdfi_timing_enable(1 if on else 0)


def timing_read(names=("sweep", "resolve", "certify", "greedy", "witness", "rmin")):
    """{name: (total ms, launches)} recorded since timing() was enabled."""
    out = {}
    for nm in names:
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib().sdfi_timing_query(nm.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "sdfi_timing_query")
        out[nm] = (ms.value, cnt.value)
    return out


def counter_read(name):
    """Work counter `name` recorded since timing() was enabled (see sdfi_counter_query)."""
    v = ctypes.c_int64()
    _check(lib().sdfi_counter_query(name.encode(), ctypes.byref(v)), "sdfi_counter_query")
    return v.value


def workspace_bytes(op, n, m, opt):
    size = ctypes.c_size_t()
    _check(lib().sdfi_workspace_size(op, n, m, ctypes.byref(opt), ctypes.byref(size)), "sdfi_workspace_size")
    return int(size.value)


def workspace(op, n, m, opt, extra=0):
    return torch.empty(max(workspace_bytes(op, n, m, opt) + extra, 256), dtype=torch.uint8, device="cuda")


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


def bounds_noalloc(samples, queries, precision="fp32"):
    """sdfi_bounds through the entry point that allocates nothing (its
    workspace is the library's scratch array; sizes are limited)."""
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
    _check(lib().sdfi_bounds_noalloc(_ptr(samples), ctypes.c_int64(n), _ptr(queries), ctypes.c_int64(m), _ptr(lo),
                                     _ptr(hi), _ptr(a), _ptr(b), _ptr(f), ctypes.byref(opt), _stream()),
           "sdfi_bounds_noalloc")
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


def refinement_order(samples, grid, queries=None):
    """Refinement order (int64 query indices)."""
    samples = _dev(samples, torch.float64, 4, "samples")
    n = samples.shape[0]
    m = 8 * n if queries is None else queries.shape[0]
    if queries is not None:
        queries = _dev(queries, torch.float64, 3, "queries")
    opt = options(grid=grid)
    out = torch.empty(m, dtype=torch.int64, device=samples.device)
    ws = workspace(OP_ORDER, n, m, opt)
    _check(lib().sdfi_refinement_order(_ptr(samples), ctypes.c_int64(n), _ptr(queries), ctypes.c_int64(m),
                                       _ptr(out), _ptr(ws), ctypes.c_size_t(ws.numel()), ctypes.byref(opt),
                                       _stream()), "sdfi_refinement_order")
    return out


def sample_witnesses(samples):
    samples = _dev(samples, torch.float64, 4, "samples")
    n = samples.shape[0]
    opt = options()
    w = torch.empty((n, 3), dtype=torch.float64, device=samples.device)
    st = torch.empty(n, dtype=torch.uint8, device=samples.device)
    ws = workspace(OP_WITNESS, n, 0, opt)
    _check(lib().sdfi_sample_witnesses(_ptr(samples), ctypes.c_int64(n), _ptr(w), _ptr(st), _ptr(ws),
                                       ctypes.c_size_t(ws.numel()), ctypes.byref(opt), _stream()),
           "sdfi_sample_witnesses")
    return w, st


def greedy(samples, queries, order=None, grid=0, certify=False, input_check=False, sample_witness=False,
           block_size=0, exhaustive=False, groups=0):
    """Greedy interpolation.  Returns a dict of GPU tensors and the host report.
    exhaustive: the exact searches take their last-resort rim walk (testing)."""
    samples = _dev(samples, torch.float64, 4, "samples")
    queries = _dev(queries, torch.float64, 3, "queries")
    n, m = samples.shape[0], queries.shape[0]
    flags = (OPT_CERTIFY if certify else 0) | (OPT_INPUT_CHECK if input_check else 0)
    flags |= OPT_EXHAUSTIVE if exhaustive else 0
    opt = options(grid=grid, flags=flags, block_size=block_size, groups=groups)
    dev = samples.device
    if order is not None:
        order = _dev(order, torch.int64, None, "order")
    out = {
        "values": torch.empty(m, dtype=torch.float64, device=dev),
        "order": torch.empty(m, dtype=torch.int64, device=dev),
        "active": torch.empty(m, dtype=torch.int64, device=dev),
        "kind": torch.empty(m, dtype=torch.uint8, device=dev),
        "witness": torch.empty((m, 3), dtype=torch.float64, device=dev),
        "sample_witness": torch.empty((n, 3), dtype=torch.float64, device=dev) if sample_witness else None,
    }
    rep = Report()
    ws = workspace(OP_GREEDY, n, m, opt)
    _check(lib().sdfi_greedy_interpolate(
        _ptr(samples), ctypes.c_int64(n), _ptr(queries), ctypes.c_int64(m), _ptr(order), _ptr(out["values"]),
        _ptr(out["order"]), _ptr(out["active"]), _ptr(out["kind"]), _ptr(out["witness"]),
        _ptr(out["sample_witness"]), ctypes.byref(rep), _ptr(ws), ctypes.c_size_t(ws.numel()), ctypes.byref(opt),
        _stream()), "sdfi_greedy_interpolate")
    out["report"] = rep.as_dict()
    return out


def greedy_batched(instances, certify=False, block_size=0, groups=0):
    """instances: list of (samples (n_i,4), queries (8 n_i,3), grid_i) GPU tensors.
    groups: most work-groups per instance (0: 16); the resident groups are shared
    out by pair count when there are at least two per instance."""
    soff = [0]
    qoff = [0]
    for s, q, g in instances:
        soff.append(soff[-1] + s.shape[0])
        qoff.append(qoff[-1] + q.shape[0])
    samples = torch.cat([_dev(s, torch.float64, 4, "samples") for s, _, _ in instances])
    queries = torch.cat([_dev(q, torch.float64, 3, "queries") for _, q, _ in instances])
    grids = (ctypes.c_int32 * len(instances))(*[int(g) for _, _, g in instances])
    so = (ctypes.c_int64 * len(soff))(*soff)
    qo = (ctypes.c_int64 * len(qoff))(*qoff)
    n, m = soff[-1], qoff[-1]
    opt = options(flags=OPT_CERTIFY if certify else 0, block_size=block_size, groups=groups)
    dev = samples.device
    out = {
        "values": torch.empty(m, dtype=torch.float64, device=dev),
        "order": torch.empty(m, dtype=torch.int64, device=dev),
        "active": torch.empty(m, dtype=torch.int64, device=dev),
        "kind": torch.empty(m, dtype=torch.uint8, device=dev),
        "witness": torch.empty((m, 3), dtype=torch.float64, device=dev),
        "sample_offsets": soff, "query_offsets": qoff,
    }
    rep = Report()
    ws = workspace(OP_GREEDY, n + len(instances), m, opt,
                   extra=len(instances) * workspace_bytes(OP_GREEDY_INSTANCE, 0, 0, opt))
    _check(lib().sdfi_greedy_interpolate_batched(
        ctypes.c_int32(len(instances)), so, qo, grids, _ptr(samples), _ptr(queries), _ptr(out["values"]),
        _ptr(out["order"]), _ptr(out["active"]), _ptr(out["kind"]), _ptr(out["witness"]), ctypes.byref(rep),
        _ptr(ws), ctypes.c_size_t(ws.numel()), ctypes.byref(opt), _stream()), "sdfi_greedy_interpolate_batched")
    out["report"] = rep.as_dict()
    return out


def min_valid_radius(samples, queries):
    """Minimum valid radius (sign by containment) of each query point."""
    samples = _dev(samples, torch.float64, 4, "samples")
    queries = _dev(queries, torch.float64, 3, "queries")
    n, m = samples.shape[0], queries.shape[0]
    opt = options()
    dev = samples.device
    val = torch.empty(m, dtype=torch.float64, device=dev)
    kind = torch.empty(m, dtype=torch.uint8, device=dev)
    wit = torch.empty((m, 3), dtype=torch.float64, device=dev)
    ws = workspace(OP_RMIN, n, m, opt)
    _check(lib().sdfi_min_valid_radius(_ptr(samples), ctypes.c_int64(n), _ptr(queries), ctypes.c_int64(m),
                                       _ptr(val), _ptr(kind), _ptr(wit), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                       ctypes.byref(opt), _stream()), "sdfi_min_valid_radius")
    return val, kind, wit


def repair(samples, queries=None):
    """Pseudo-SDF repair.  Returns (repaired values, removed mask, query values, kinds, report)."""
    samples = _dev(samples, torch.float64, 4, "samples")
    dev = samples.device
    if queries is None:
        queries = torch.zeros((0, 3), dtype=torch.float64, device=dev)
    queries = _dev(queries, torch.float64, 3, "queries")
    n, m = samples.shape[0], queries.shape[0]
    opt = options()
    rep_v = torch.empty(n, dtype=torch.float64, device=dev)
    removed = torch.empty(n, dtype=torch.uint8, device=dev)
    qv = torch.empty(max(m, 1), dtype=torch.float64, device=dev)
    kind = torch.empty(n + m, dtype=torch.uint8, device=dev)
    rep = Report()
    ws = workspace(OP_REPAIR, n, m, opt)
    _check(lib().sdfi_repair(_ptr(samples), ctypes.c_int64(n), _ptr(queries), ctypes.c_int64(m), _ptr(rep_v),
                             _ptr(removed), _ptr(qv), _ptr(kind), ctypes.byref(rep), _ptr(ws),
                             ctypes.c_size_t(ws.numel()), ctypes.byref(opt), _stream()), "sdfi_repair")
    return rep_v, removed, qv[:m], kind, rep.as_dict()


def greedy_backward(grad_values, samples, queries, values, active, kind):
    """d(sum grad_values * values)/d(sample values, sample positions)."""
    samples = _dev(samples, torch.float64, 4, "samples")
    queries = _dev(queries, torch.float64, 3, "queries")
    grad_values = _dev(grad_values, torch.float64, None, "grad_values")
    values = _dev(values, torch.float64, None, "values")
    active = _dev(active, torch.int64, None, "active")
    kind = _dev(kind, torch.uint8, None, "kind")
    n, m = samples.shape[0], queries.shape[0]
    gs = torch.empty(n, dtype=torch.float64, device=samples.device)
    gp = torch.empty((n, 3), dtype=torch.float64, device=samples.device)
    ws = workspace(OP_BACKWARD, n, m, options())
    _check(lib().sdfi_greedy_backward(_ptr(grad_values), _ptr(samples), ctypes.c_int64(n), _ptr(queries),
                                      ctypes.c_int64(m), _ptr(values), _ptr(active), _ptr(kind), _ptr(gs), _ptr(gp),
                                      _ptr(ws), ctypes.c_size_t(ws.numel()), _stream()), "sdfi_greedy_backward")
    return gs, gp


class GreedyInterpolate(torch.autograd.Function):
    """values = greedy interpolation of `queries` from samples (points, values).

    Forward runs sdfi_greedy_interpolate; backward runs sdfi_greedy_backward,
    the adjoint through each value's active parent (decisions held fixed).
    Gradients flow to the sample positions (n, 3) and values (n,).
    """

    @staticmethod
    def forward(ctx, points, values, queries, grid=0, order=None):
        samples = torch.cat([points.detach(), values.detach()[:, None]], dim=1).contiguous()
        out = greedy(samples, queries.detach(), order=order, grid=grid)
        ctx.save_for_backward(samples, queries.detach(), out["values"], out["active"], out["kind"])
        ctx.mark_non_differentiable(out["kind"], out["active"])
        return out["values"], out["kind"], out["active"]

    @staticmethod
    def backward(ctx, gv, _gk=None, _ga=None):
        samples, queries, values, active, kind = ctx.saved_tensors
        gs, gp = greedy_backward(gv.contiguous().to(torch.float64), samples, queries, values, active, kind)
        return gp, gs, None, None, None
