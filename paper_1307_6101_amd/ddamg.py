"""Thin ctypes binding of libddamg.so (C ABI in include/ddamg.h).

Argument marshalling only: tensors are passed as device pointers
(``tensor.data_ptr()``) together with torch's current HIP stream; every
computation runs in the library's kernels.  The functions keep the names of
the C entry points without the ``ddamg_`` prefix.  Importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddamg.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
F64, F32, F16, F16S = 0, 1, 2, 3
CANONICAL, NATIVE = 0, 1
KCYCLE, VCYCLE, WCYCLE = 0, 1, 2


class DDAMGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ddamg error {status}: {msg}")
        self.status = status


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("m0", ctypes.c_double), ("csw", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int),
        ("agg", (ctypes.c_int * 4) * 3),
        ("ntv", ctypes.c_int * 3),
        ("sap_block", ctypes.c_int * 4),
        ("mu", ctypes.c_int), ("nu", ctypes.c_int),
        ("mr_iters", ctypes.c_int),
        ("n_inv", ctypes.c_int),
        ("coarse_eps", ctypes.c_double),
        ("coarse_restart", ctypes.c_int),
        ("coarse_max_restarts", ctypes.c_int),
        ("kc_len", ctypes.c_int),
        ("kc_restarts", ctypes.c_int),
        ("kc_tol", ctypes.c_double),
        ("nkv", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_restarts", ctypes.c_int),
        ("precond_prec", ctypes.c_int),
        ("cycle", ctypes.c_int),
        ("half_storage", ctypes.c_int),
        ("batch", ctypes.c_int),
        ("sap_block_l", (ctypes.c_int * 4) * 3),
        ("half_directions", ctypes.c_int),
        ("graph", ctypes.c_int),
        ("coarse_dense", ctypes.c_int),
        ("galerkin_cols", ctypes.c_int),
        ("profile_levels", ctypes.c_int),
        ("half_spinors", ctypes.c_int),
    ]


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("outer_iters", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("kcycle_iters", ctypes.c_longlong),
        ("coarsest_iters", ctypes.c_longlong),
        ("true_relres", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("err_vs_ref", ctypes.c_double),
        ("t_setup_s", ctypes.c_double),
        ("t_level_s", ctypes.c_double * 4),
        ("bytes", ctypes.c_double),
        ("flops", ctypes.c_double),
        ("coarsest_dense", ctypes.c_int),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["t_level_s"] = list(self.t_level_s)
        return d


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("sap_block_l", (ctypes.c_int * 4) * 3),
        ("batch", ctypes.c_int),
        ("seconds", ctypes.c_double),
        ("from_cache", ctypes.c_int),
    ]


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "ddamg_params_default": (None, [ctypes.POINTER(Params), _I]),
    "ddamg_last_error": (ctypes.c_char_p, []),
    "ddamg_version": (ctypes.c_char_p, []),
    "ddamg_create": (_I, [ctypes.POINTER(Lattice), _P, _P, ctypes.POINTER(_P)]),
    "ddamg_workspace_bytes": (_I, [ctypes.POINTER(Lattice), ctypes.POINTER(Params), _I,
                                   ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "ddamg_create_ws": (_I, [ctypes.POINTER(Lattice), _P, ctypes.POINTER(Params), _I, _P, ctypes.c_size_t, _P,
                             ctypes.POINTER(_P)]),
    "ddamg_destroy": (None, [_P]),
    "ddamg_apply_D": (_I, [_P, _P, _P, _I, _I, _I, _P]),
    "ddamg_apply_D_noalloc": (_I, [_P, _P, _P, _I, _I, _P]),
    "ddamg_to_native": (_I, [_P, _P, _I, _P, _P, _I, _I, _P]),
    "ddamg_from_native": (_I, [_P, _P, _I, _P, _P, _I, _I, _P]),
    "ddamg_build_hierarchy": (_I, [_P, ctypes.POINTER(Params), _P, _P, _P, ctypes.POINTER(_P)]),
    "ddamg_build_hierarchy_ws": (_I, [_P, ctypes.POINTER(Params), _P, _P, _I, _P, ctypes.c_size_t, _P,
                                      ctypes.POINTER(_P)]),
    "ddamg_destroy_hierarchy": (None, [_P]),
    "ddamg_level_info": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int * 4), ctypes.POINTER(_I)]),
    "ddamg_apply_Dc": (_I, [_P, _I, _P, _P, _I, _I, _I, _P]),
    "ddamg_restrict": (_I, [_P, _I, _P, _P, _I, _I, _I, _P]),
    "ddamg_prolong": (_I, [_P, _I, _P, _P, _I, _I, _I, _P]),
    "ddamg_sap_smooth": (_I, [_P, _I, _P, _P, _I, _I, _I, _I, _P]),
    "ddamg_precondition": (_I, [_P, _P, _P, _I, _I, _P]),
    "ddamg_solve": (_I, [_P, _P, _P, _I, ctypes.POINTER(SolveStats), _P]),
    "ddamg_solve_ex": (_I, [_P, _P, _P, _I, _P, ctypes.POINTER(SolveStats), _P]),
    "ddamg_solve_many": (_I, [_I, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                              ctypes.POINTER(_I), ctypes.POINTER(SolveStats), _P]),
    "ddamg_solve_batch": (_I, [_I, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                               ctypes.POINTER(SolveStats), _P]),
    "ddamg_set_sap_block": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int * 4)]),
    "ddamg_set_batch": (_I, [_P, _I]),
    "ddamg_tune": (_I, [_P, _P, _I, ctypes.c_char_p, ctypes.POINTER(TuneResult), _P]),
    "ddamg_cgnr": (_I, [_P, _P, _P, _I, ctypes.c_double, _I, ctypes.POINTER(SolveStats), _P]),
    "ddamg_export_interpolation": (_I, [_P, _I, _P, _P]),
    "ddamg_export_coarse_op": (_I, [_P, _I, _P, _P]),
    "ddamg_import_test_vectors": (_I, [_P, _I, _P, _P]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libddamg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (paper_1307_6101_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise DDAMGError(rc, load_library().ddamg_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensors only")
    if not t.is_contiguous():
        raise ValueError("contiguous tensors only")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def version() -> str:
    return load_library().ddamg_version().decode()


def params_default(levels: int) -> Params:
    p = Params()
    load_library().ddamg_params_default(ctypes.byref(p), levels)
    return p


def _ws(t):
    """A workspace tensor: contiguous device bytes."""
    if t.dtype != torch.uint8:
        raise ValueError("a workspace is a torch.uint8 device tensor")
    return _ptr(t), ctypes.c_size_t(t.numel())


def workspace_bytes(dims, m0, csw, params=None, nrhs_max=1):
    """(context bytes, hierarchy bytes) of ddamg_workspace_bytes; the second
    is 0 without params."""
    lib = load_library()
    lat = Lattice((ctypes.c_int * 4)(*dims), float(m0), float(csw))
    cb, hb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _check(lib.ddamg_workspace_bytes(ctypes.byref(lat), ctypes.byref(params) if params is not None else None,
                                     int(nrhs_max), ctypes.byref(cb), ctypes.byref(hb)))
    return cb.value, hb.value


class Context:
    """Handle of one lattice operator D (ddamg_create / ddamg_destroy); with
    `workspace` (a torch.uint8 device tensor) ddamg_create_ws, which keeps
    all of the handle's device memory in that tensor (held here until the
    handle is destroyed)."""

    def __init__(self, dims, m0, csw, links, workspace=None, params=None, nrhs_max=1):
        lib = load_library()
        lat = Lattice((ctypes.c_int * 4)(*dims), float(m0), float(csw))
        h = ctypes.c_void_p()
        if workspace is None:
            _check(lib.ddamg_create(ctypes.byref(lat), _ptr(links), _stream(), ctypes.byref(h)))
        else:
            wp, wn = _ws(workspace)
            _check(lib.ddamg_create_ws(ctypes.byref(lat), _ptr(links),
                                       ctypes.byref(params) if params is not None else None, int(nrhs_max),
                                       wp, wn, _stream(), ctypes.byref(h)))
        self.handle = h
        self.dims = tuple(dims)
        self.workspace = workspace

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ddamg_destroy(self.handle)
            self.handle = None


class Hierarchy:
    """Handle of a multilevel hierarchy (ddamg_build_hierarchy / destroy);
    with `workspace` ddamg_build_hierarchy_ws (see Context)."""

    def __init__(self, ctx: Context, params: Params, tv, tv_extra=None, workspace=None, nrhs_max=1):
        lib = load_library()
        h = ctypes.c_void_p()
        if workspace is None:
            _check(lib.ddamg_build_hierarchy(ctx.handle, ctypes.byref(params), _ptr(tv), _ptr(tv_extra),
                                             _stream(), ctypes.byref(h)))
        else:
            wp, wn = _ws(workspace)
            _check(lib.ddamg_build_hierarchy_ws(ctx.handle, ctypes.byref(params), _ptr(tv), _ptr(tv_extra),
                                                int(nrhs_max), wp, wn, _stream(), ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx
        self.params = params
        self.workspace = workspace

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ddamg_destroy_hierarchy(self.handle)
            self.handle = None


def create(dims, m0, csw, links) -> Context:
    return Context(dims, m0, csw, links)


def build_hierarchy(ctx, params, tv, tv_extra=None) -> Hierarchy:
    return Hierarchy(ctx, params, tv, tv_extra)


def create_ws(dims, m0, csw, links, workspace, params=None, nrhs_max=1) -> Context:
    return Context(dims, m0, csw, links, workspace=workspace, params=params, nrhs_max=nrhs_max)


def build_hierarchy_ws(ctx, params, tv, workspace, nrhs_max=1, tv_extra=None) -> Hierarchy:
    return Hierarchy(ctx, params, tv, tv_extra, workspace=workspace, nrhs_max=nrhs_max)


def apply_D(ctx, inp, out, nrhs=1, prec=F64, layout=CANONICAL):
    _check(load_library().ddamg_apply_D(ctx.handle, _ptr(inp), _ptr(out), nrhs, prec, layout, _stream()))


def apply_D_noalloc(ctx, inp, out, nrhs=1, prec=F64):
    """ddamg_apply_D_noalloc: canonical out = D inp through the library's
    fixed device staging array (no allocation)."""
    _check(load_library().ddamg_apply_D_noalloc(ctx.handle, _ptr(inp), _ptr(out), nrhs, prec, _stream()))


NOALLOC_SCRATCH_BYTES = 64 << 20


def to_native(ctx, hier, level, inp, out, nrhs=1, prec=F64):
    h = hier.handle if hier is not None else None
    _check(load_library().ddamg_to_native(ctx.handle, h, level, _ptr(inp), _ptr(out), nrhs, prec, _stream()))


def from_native(ctx, hier, level, inp, out, nrhs=1, prec=F64):
    h = hier.handle if hier is not None else None
    _check(load_library().ddamg_from_native(ctx.handle, h, level, _ptr(inp), _ptr(out), nrhs, prec, _stream()))


def level_info(hier, level):
    dims = (ctypes.c_int * 4)()
    dof = ctypes.c_int()
    _check(load_library().ddamg_level_info(hier.handle, level, ctypes.byref(dims), ctypes.byref(dof)))
    return tuple(dims), dof.value


def apply_Dc(hier, level, inp, out, nrhs=1, prec=F64, layout=CANONICAL):
    _check(load_library().ddamg_apply_Dc(hier.handle, level, _ptr(inp), _ptr(out), nrhs, prec, layout,
                                         _stream()))


def restrict(hier, level, fine, coarse, nrhs=1, prec=F64, layout=CANONICAL):
    _check(load_library().ddamg_restrict(hier.handle, level, _ptr(fine), _ptr(coarse), nrhs, prec, layout,
                                         _stream()))


def prolong(hier, level, coarse, fine, nrhs=1, prec=F64, layout=CANONICAL):
    _check(load_library().ddamg_prolong(hier.handle, level, _ptr(coarse), _ptr(fine), nrhs, prec, layout,
                                        _stream()))


def sap_smooth(hier, level, b, z, nsweeps, nrhs=1, prec=F64, layout=CANONICAL):
    _check(load_library().ddamg_sap_smooth(hier.handle, level, _ptr(b), _ptr(z), nsweeps, nrhs, prec,
                                           layout, _stream()))


def precondition(hier, b, z, nrhs=1, layout=CANONICAL):
    _check(load_library().ddamg_precondition(hier.handle, _ptr(b), _ptr(z), nrhs, layout, _stream()))


def solve(hier, b, z, nrhs=1):
    """Solve D z = b; returns (status, [stats dict per right-hand side]).
    ENOCONV / ENONFINITE are returned, other failures raise."""
    stats = (SolveStats * nrhs)()
    rc = load_library().ddamg_solve(hier.handle, _ptr(b), _ptr(z), nrhs, stats, _stream())
    if rc not in (OK, ENOCONV, ENONFINITE):
        _check(rc)
    return rc, [s.as_dict() for s in stats]


def solve_ex(hier, b, z, z_ref=None, nrhs=1):
    """ddamg_solve_ex: solve D z = b and, with z_ref, report each system's
    error ||z - z_ref|| / ||z_ref||; returns (status, [stats dicts])."""
    stats = (SolveStats * nrhs)()
    rc = load_library().ddamg_solve_ex(hier.handle, _ptr(b), _ptr(z), nrhs, _ptr(z_ref), stats, _stream())
    if rc not in (OK, ENOCONV, ENONFINITE):
        _check(rc)
    return rc, [s.as_dict() for s in stats]


def solve_many(hiers, bs, zs, nrhs=None):
    """Solve the independent systems hiers[i]: D z_i = b_i concurrently (the
    hierarchies may belong to lattices of different sizes); returns (status,
    [stats dicts of system 0's right-hand sides, then system 1's, ...]).
    ENOCONV / ENONFINITE are returned, other failures raise."""
    n = len(hiers)
    if len(bs) != n or len(zs) != n:
        raise ValueError("one b and one z per hierarchy")
    nrhs = [1] * n if nrhs is None else list(nrhs)
    hv = (_P * n)(*[h.handle for h in hiers])
    bv = (_P * n)(*[_ptr(b) for b in bs])
    zv = (_P * n)(*[_ptr(z) for z in zs])
    nv = (_I * n)(*nrhs)
    stats = (SolveStats * max(1, sum(nrhs)))()
    rc = load_library().ddamg_solve_many(n, hv, bv, zv, nv, stats, _stream())
    if rc not in (OK, ENOCONV, ENONFINITE):
        _check(rc)
    return rc, [s.as_dict() for s in stats[:sum(nrhs)]]


def solve_batch(hiers, bs, zs):
    """The uneven batch as one graph per outer step (ddamg_solve_batch): one
    right-hand side per hierarchy; returns (status, [stats dict per system]).
    ENOCONV / ENONFINITE are returned, other failures raise."""
    n = len(hiers)
    if len(bs) != n or len(zs) != n:
        raise ValueError("one b and one z per hierarchy")
    hv = (_P * n)(*[h.handle for h in hiers])
    bv = (_P * n)(*[_ptr(b) for b in bs])
    zv = (_P * n)(*[_ptr(z) for z in zs])
    stats = (SolveStats * n)()
    rc = load_library().ddamg_solve_batch(n, hv, bv, zv, stats, _stream())
    if rc not in (OK, ENOCONV, ENONFINITE):
        _check(rc)
    return rc, [s.as_dict() for s in stats]


def set_sap_block(hier, level, block):
    _check(load_library().ddamg_set_sap_block(hier.handle, level, ctypes.byref((ctypes.c_int * 4)(*block))))


def set_batch(hier, batch):
    _check(load_library().ddamg_set_batch(hier.handle, batch))


def tune(hier, b, nrhs=1, cache=None):
    """Autotune the coarse SAP block shapes and the batch size by timing
    solves of b (applied to the hierarchy); returns a dict of the choice."""
    r = TuneResult()
    path = None if cache is None else os.fspath(cache).encode()
    _check(load_library().ddamg_tune(hier.handle, _ptr(b), nrhs, path, ctypes.byref(r), _stream()))
    return dict(sap_block_l=[list(row) for row in r.sap_block_l], batch=r.batch, seconds=r.seconds,
                from_cache=bool(r.from_cache))


def cgnr(ctx, b, z, nrhs=1, tol=1e-10, max_iter=100000):
    """CGNR in FP64 on the context's operator; returns (status, [stats
    dicts]), outer_iters holding the CG iteration count.  ENOCONV /
    ENONFINITE are returned, other failures raise."""
    stats = (SolveStats * nrhs)()
    rc = load_library().ddamg_cgnr(ctx.handle, _ptr(b), _ptr(z), nrhs, tol, max_iter, stats, _stream())
    if rc not in (OK, ENOCONV, ENONFINITE):
        _check(rc)
    return rc, [s.as_dict() for s in stats]


def export_interpolation(hier, level, out):
    _check(load_library().ddamg_export_interpolation(hier.handle, level, _ptr(out), _stream()))


def export_coarse_op(hier, level, out):
    _check(load_library().ddamg_export_coarse_op(hier.handle, level, _ptr(out), _stream()))


def import_test_vectors(hier, level, tv):
    _check(load_library().ddamg_import_test_vectors(hier.handle, level, _ptr(tv), _stream()))
