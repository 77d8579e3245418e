"""Refined-wall Stokes solver for AMD MI355X (gfx950): Python binding.

Thin ctypes marshalling over the C ABI in ``include/rw.h`` (``librw.so``,
built by ``python -m paper_2108_07205_amd.build``).  Every step of the solve
runs in the library's HIP kernels; PyTorch only provides device memory and
the HIP stream.  The module-level functions carry the C names
(``rw_ctx_create``, ``rw_wall_build``, ``rw_refine``, ``rw_solve`` ...); the
``Context`` / ``Wall`` / ``Refined`` classes are small conveniences on top.

Importing this package never falls back to anything: if ``librw.so`` is
missing, ``load_library()`` raises.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "RwError", "load_library", "Context", "Wall", "Refined",
    "rw_ctx_create", "rw_ctx_destroy", "rw_set_options", "rw_get_options", "rw_wall_build",
    "rw_wall_free", "rw_wall_stats_get", "rw_wall_nodes", "rw_hbs_apply", "rw_hbs_apply_noalloc", "rw_refine",
    "rw_coarsen",
    "rw_refined_free", "rw_refined_info", "rw_nodes", "rw_solve", "rw_residual", "rw_stokeslet_rhs",
    "rw_ctx_trim", "rw_profile_enable", "rw_profile_reset", "rw_profile_json",
    "RW_OK", "RW_EINVAL", "RW_ENOMEM", "RW_ESINGULAR", "RW_ENOCONV", "RW_EDEVICE", "RW_F64", "RW_F32",
    "RW_BF16", "RW_SOLVE_IR", "RW_SOLVE_GMRES", "RW_RESID_AUTO", "RW_RESID_PAIRS", "RW_RESID_EXPAND",
    "rw_solve_batch", "rw_refine_on", "Server", "RefCache",
    "EXPORTED_SYMBOLS",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librw.so")

RW_OK, RW_EINVAL, RW_ENOMEM, RW_ESINGULAR, RW_ENOCONV, RW_EDEVICE = 0, -1, -2, -3, -4, -5
RW_F64, RW_F32, RW_BF16 = 0, 1, 2
RW_SOLVE_IR, RW_SOLVE_GMRES = 0, 1
RW_RESID_AUTO, RW_RESID_PAIRS, RW_RESID_EXPAND = 0, 1, 2
_CODES = {RW_EINVAL: "RW_EINVAL", RW_ENOMEM: "RW_ENOMEM", RW_ESINGULAR: "RW_ESINGULAR",
          RW_ENOCONV: "RW_ENOCONV", RW_EDEVICE: "RW_EDEVICE"}


class RwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class rw_curve(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("m", ctypes.c_int32)]


class rw_options(ctypes.Structure):
    _fields_ = [("ir_tol", ctypes.c_double), ("ir_maxit", ctypes.c_int32),
                ("sketch_cols", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("app_dense_max_nodes", ctypes.c_int32), ("far_field", ctypes.c_int32),
                ("hbs_merge", ctypes.c_int32), ("solver", ctypes.c_int32), ("gmres_restart", ctypes.c_int32),
                ("gmres_precond", ctypes.c_int32), ("mfma_from", ctypes.c_int32), ("test_singular", ctypes.c_int32),
                ("one_stream", ctypes.c_int32),
                ("resid_mode", ctypes.c_int32)]


class rw_info(ctypes.Structure):
    _fields_ = [("n_k", ctypes.c_int64), ("n_c", ctypes.c_int64), ("n_p", ctypes.c_int64),
                ("k_k", ctypes.c_int32), ("k_p", ctypes.c_int32), ("k", ctypes.c_int32),
                ("ir_iters", ctypes.c_int32), ("resid", ctypes.c_double),
                ("t_refine_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double), ("n_near", ctypes.c_int64),
                ("app_entries", ctypes.c_int64), ("app_max_rank", ctypes.c_int32),
                ("app_lu_mult", ctypes.c_double)]


class rw_solve_info(ctypes.Structure):
    _fields_ = [("ir_iters", ctypes.c_int32), ("k", ctypes.c_int32), ("resid", ctypes.c_double),
                ("resid_direct", ctypes.c_double), ("t_solve_ms", ctypes.c_double)]


class rw_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("ir_iters", ctypes.c_int32),
                ("k", ctypes.c_int32), ("n_nodes", ctypes.c_int64), ("resid", ctypes.c_double),
                ("t_queue_ms", ctypes.c_double), ("t_run_ms", ctypes.c_double)]


class rw_wall_stats(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_levels", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("gen_entries", ctypes.c_int64), ("gen_bytes_f64", ctypes.c_int64),
                ("t_build_ms", ctypes.c_double), ("mfma_from_f64", ctypes.c_int32),
                ("mfma_from_f32", ctypes.c_int32)]


_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_DP = ctypes.POINTER(ctypes.c_double)
_I64P = ctypes.POINTER(ctypes.c_int64)

# symbol -> (restype, argtypes); the set of exported C functions of rw.h
_SIGS = {
    "rw_ctx_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, ctypes.c_size_t]),
    "rw_ctx_destroy": (None, [_P]),
    "rw_last_error": (ctypes.c_char_p, [_P]),
    "rw_create_error": (ctypes.c_char_p, []),
    "rw_set_options": (ctypes.c_int, [_P, ctypes.POINTER(rw_options)]),
    "rw_get_options": (ctypes.c_int, [_P, ctypes.POINTER(rw_options)]),
    "rw_ctx_bytes": (ctypes.c_size_t, [_P]),
    "rw_ctx_trim": (ctypes.c_int, [_P]),
    "rw_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "rw_profile_reset": (ctypes.c_int, [_P]),
    "rw_profile_json": (ctypes.c_int64, [_P, ctypes.c_char_p, ctypes.c_int64]),
    "rw_wall_build": (ctypes.c_int, [_P, ctypes.POINTER(rw_curve), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_P)]),
    "rw_wall_free": (None, [_P]),
    "rw_wall_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(rw_wall_stats)]),
    "rw_wall_nodes": (ctypes.c_int, [_P, _DP, _DP, _DP, _I64P]),
    "rw_hbs_apply": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P]),
    "rw_hbs_apply_noalloc": (ctypes.c_int, [_P, _P, _P]),
    "rw_refine": (ctypes.c_int, [_P, _I32P, _I32P, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_P)]),
    "rw_coarsen": (ctypes.c_int, [_P, _I32P, ctypes.c_int32]),
    "rw_refined_free": (None, [_P]),
    "rw_refined_info": (ctypes.c_int, [_P, ctypes.POINTER(rw_info)]),
    "rw_nodes": (ctypes.c_int, [_P, _DP, _DP, _DP, _I64P]),
    "rw_solve": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.POINTER(rw_solve_info)]),
    "rw_solve_batch": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "rw_residual": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P]),
    "rw_stokeslet_rhs": (ctypes.c_int, [_P, _DP, _DP, ctypes.c_int32, _P]),
    "rw_refine_on": (ctypes.c_int, [_P, _P, _I32P, _I32P, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_P)]),
    "rw_server_create": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "rw_server_submit": (ctypes.c_int, [_P, _I32P, _I32P, ctypes.c_int32, _DP, _DP, ctypes.c_int32, ctypes.c_int32,
                                        _I64P]),
    "rw_server_wait": (ctypes.c_int, [_P, ctypes.c_int64, _DP, ctypes.c_int64, ctypes.POINTER(rw_request_info)]),
    "rw_server_destroy": (None, [_P]),
    "rw_server_error": (ctypes.c_char_p, [_P]),
    "rw_refcache_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                          ctypes.POINTER(_P)]),
    "rw_refcache_get": (ctypes.c_int, [_P, _I32P, _I32P, ctypes.c_int32, ctypes.POINTER(_P), _I32P]),
    "rw_refcache_panels": (ctypes.c_int, [_P, _P, _I32P, _I32P, _I32P]),
    "rw_refcache_stats": (None, [_P, _I64P, _I64P, _I32P]),
    "rw_refcache_destroy": (None, [_P]),
    "rw_refcache_error": (ctypes.c_char_p, [_P]),
}
EXPORTED_SYMBOLS = tuple(_SIGS)

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``librw.so`` (raises if it has not been built).  PyTorch is
    imported first: it brings a HIP runtime of its own, and the library must
    bind to that one (a second runtime loaded beside it finds no device)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2108_07205_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, ctx=None):
    if rc != RW_OK:
        lib = load_library()
        msg = lib.rw_last_error(ctx).decode() if ctx else lib.rw_create_error().decode()
        raise RwError(rc, msg)


def _dev_ptr(t, name: str, rows: int = None):
    """Pointer and column count of a contiguous float64 device tensor of shape
    (rows,) or (ncols, rows) (= column-major rows x ncols)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dim() == 1:
        n, ncols = t.shape[0], 1
    elif t.dim() == 2:
        ncols, n = t.shape
    else:
        raise ValueError(f"{name} must be 1-D or 2-D")
    if rows is not None and n != rows:
        raise ValueError(f"{name} has {n} rows, expected {rows}")
    return ctypes.c_void_p(t.data_ptr()), int(ncols)


# ----------------------------------------------------------------- C names
def rw_ctx_create(device: int = 0, stream: Optional[int] = None, hbm_budget_bytes: int = 0):
    lib = load_library()
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(device).cuda_stream
    out = _P()
    _check(lib.rw_ctx_create(ctypes.byref(out), device, _P(stream), hbm_budget_bytes))
    return out


def rw_ctx_destroy(ctx):
    load_library().rw_ctx_destroy(ctx)


def rw_set_options(ctx, ir_tol=None, ir_maxit=None, sketch_cols=None, seed=None, app_dense_max_nodes=None,
                   far_field=None, test_singular=None, hbs_merge=None, solver=None, gmres_restart=None,
                   gmres_precond=None, mfma_from=None, one_stream=None, resid_mode=None):
    lib = load_library()
    o = rw_options()
    _check(lib.rw_get_options(ctx, ctypes.byref(o)), ctx)
    if ir_tol is not None:
        o.ir_tol = ir_tol
    if ir_maxit is not None:
        o.ir_maxit = ir_maxit
    if sketch_cols is not None:
        o.sketch_cols = sketch_cols
    if seed is not None:
        o.seed = seed
    if app_dense_max_nodes is not None:
        o.app_dense_max_nodes = app_dense_max_nodes
    if far_field is not None:
        o.far_field = int(bool(far_field))
    if test_singular is not None:
        o.test_singular = int(test_singular)
    if hbs_merge is not None:
        o.hbs_merge = int(hbs_merge)
    if solver is not None:
        o.solver = int(solver)
    if gmres_restart is not None:
        o.gmres_restart = int(gmres_restart)
    if gmres_precond is not None:
        o.gmres_precond = int(gmres_precond)
    if mfma_from is not None:
        o.mfma_from = int(mfma_from)
    if one_stream is not None:
        o.one_stream = int(bool(one_stream))
    if resid_mode is not None:
        o.resid_mode = int(resid_mode)
    _check(lib.rw_set_options(ctx, ctypes.byref(o)), ctx)


def rw_get_options(ctx) -> dict:
    o = rw_options()
    _check(load_library().rw_get_options(ctx, ctypes.byref(o)), ctx)
    return {f: getattr(o, f) for f, _ in rw_options._fields_}


def rw_ctx_trim(ctx):
    _check(load_library().rw_ctx_trim(ctx), ctx)


def rw_profile_enable(ctx, on: bool = True):
    _check(load_library().rw_profile_enable(ctx, 1 if on else 0), ctx)


def rw_profile_reset(ctx):
    _check(load_library().rw_profile_reset(ctx), ctx)


def rw_profile_json(ctx) -> dict:
    import json
    lib = load_library()
    n = lib.rw_profile_json(ctx, None, 0)
    if n < 0:
        _check(int(n), ctx)
    buf = ctypes.create_string_buffer(int(n) + 16)
    lib.rw_profile_json(ctx, buf, len(buf))
    return json.loads(buf.value.decode())


def rw_wall_build(ctx, n_panels: int, order: int = 16, leaf_nodes: int = 64, id_tol: float = 1e-10,
                  precision: int = RW_F64, a: float = 0.3, m: int = 5):
    out = _P()
    cv = rw_curve(a, m)
    _check(load_library().rw_wall_build(ctx, ctypes.byref(cv), n_panels, order, leaf_nodes, id_tol,
                                        precision, ctypes.byref(out)), ctx)
    return out


def rw_wall_free(wall):
    load_library().rw_wall_free(wall)


def rw_wall_stats_get(ctx, wall) -> dict:
    st = rw_wall_stats()
    _check(load_library().rw_wall_stats_get(wall, ctypes.byref(st)), ctx)
    return {f: getattr(st, f) for f, _ in rw_wall_stats._fields_}


def _nodes(fn, ctx, h):
    n = ctypes.c_int64(0)
    _check(fn(h, None, None, None, ctypes.byref(n)), ctx)
    xy = np.empty(2 * n.value)
    nr = np.empty(2 * n.value)
    w = np.empty(n.value)
    _check(fn(h, xy.ctypes.data_as(_DP), nr.ctypes.data_as(_DP), w.ctypes.data_as(_DP), ctypes.byref(n)), ctx)
    return xy.reshape(-1, 2), nr.reshape(-1, 2), w


def rw_wall_nodes(ctx, wall):
    return _nodes(load_library().rw_wall_nodes, ctx, wall)


def rw_hbs_apply(ctx, wall, b, x, n_unknowns: int):
    pb, nb = _dev_ptr(b, "b", n_unknowns)
    px, nx = _dev_ptr(x, "x", n_unknowns)
    if nb != nx:
        raise ValueError("b and x column counts differ")
    _check(load_library().rw_hbs_apply(wall, pb, nb, px), ctx)


def rw_hbs_apply_noalloc(ctx, wall, b, x, n_unknowns: int):
    pb, nb = _dev_ptr(b, "b", n_unknowns)
    px, nx = _dev_ptr(x, "x", n_unknowns)
    if nb != 1 or nx != 1:
        raise ValueError("rw_hbs_apply_noalloc takes one column")
    _check(load_library().rw_hbs_apply_noalloc(wall, pb, px), ctx)


def rw_refine(ctx, wall, panel_ids: Sequence[int], levels: Sequence[int], q_tol: float = 0.0):
    ids = np.ascontiguousarray(panel_ids, dtype=np.int32)
    lev = np.ascontiguousarray(levels, dtype=np.int32)
    if ids.shape != lev.shape:
        raise ValueError("panel_ids and levels differ in length")
    out = _P()
    _check(load_library().rw_refine(wall, ids.ctypes.data_as(_I32P), lev.ctypes.data_as(_I32P), ids.size,
                                    q_tol, ctypes.byref(out)), ctx)
    return out


def rw_refine_on(ctx, wall, panel_ids: Sequence[int], levels: Sequence[int], q_tol: float = 0.0):
    """rw_refine on ctx (its stream and memory) against a wall built on another ctx."""
    ids = np.ascontiguousarray(panel_ids, dtype=np.int32)
    lev = np.ascontiguousarray(levels, dtype=np.int32)
    if ids.shape != lev.shape:
        raise ValueError("panel_ids and levels differ in length")
    out = _P()
    _check(load_library().rw_refine_on(ctx, wall, ids.ctypes.data_as(_I32P), lev.ctypes.data_as(_I32P), ids.size,
                                       q_tol, ctypes.byref(out)), ctx)
    return out


def rw_coarsen(ctx, ref, panel_ids: Sequence[int]):
    ids = np.ascontiguousarray(panel_ids, dtype=np.int32)
    _check(load_library().rw_coarsen(ref, ids.ctypes.data_as(_I32P), ids.size), ctx)


def rw_refined_free(ref):
    load_library().rw_refined_free(ref)


def rw_refined_info(ctx, ref) -> dict:
    inf = rw_info()
    _check(load_library().rw_refined_info(ref, ctypes.byref(inf)), ctx)
    return {f: getattr(inf, f) for f, _ in rw_info._fields_}


def rw_nodes(ctx, ref):
    return _nodes(load_library().rw_nodes, ctx, ref)


def rw_solve(ctx, ref, g, tau, n_unknowns: int, check: bool = True, info: dict = None):
    """rc of rw_solve; when `info` is a dict it receives the rw_solve_info fields."""
    pg, ng = _dev_ptr(g, "g", n_unknowns)
    pt, nt = _dev_ptr(tau, "tau", n_unknowns)
    if ng != nt:
        raise ValueError("g and tau column counts differ")
    si = rw_solve_info()
    rc = load_library().rw_solve(ref, pg, ng, pt, ctypes.byref(si))
    if info is not None:
        info.update({f: getattr(si, f) for f, _ in rw_solve_info._fields_})
    if check:
        _check(rc, ctx)
    return rc


def rw_solve_batch(ctx, refs, gs, taus, n_unknowns, check: bool = True):
    """Marshal lists of handles and (nrhs_i, 2 N_n(i)) float64 device tensors
    into pointer arrays for the C call; returns (rc, [info dict per instance])."""
    n = len(refs)
    if not (len(gs) == len(taus) == len(n_unknowns) == n) or n == 0:
        raise ValueError("refs, gs, taus and n_unknowns must have the same non-zero length")
    hs = (_P * n)(*refs)
    pg = (_P * n)()
    pt = (_P * n)()
    nr = (ctypes.c_int32 * n)()
    for i in range(n):
        pg[i], ng = _dev_ptr(gs[i], "g", n_unknowns[i])
        pt[i], nt = _dev_ptr(taus[i], "tau", n_unknowns[i])
        if ng != nt:
            raise ValueError(f"g and tau column counts differ for instance {i}")
        nr[i] = ng
    infos = (rw_info * n)()
    rc = load_library().rw_solve_batch(hs, n, pg, nr, pt, infos)
    if check:
        _check(rc, ctx)
    return rc, [{f: getattr(inf, f) for f, _ in rw_info._fields_} for inf in infos]


def rw_residual(ctx, ref, g, tau, r, n_unknowns: int):
    pg, ng = _dev_ptr(g, "g", n_unknowns)
    pt, _ = _dev_ptr(tau, "tau", n_unknowns)
    pr, _ = _dev_ptr(r, "r", n_unknowns)
    _check(load_library().rw_residual(ref, pg, pt, ng, pr), ctx)


def rw_stokeslet_rhs(ctx, ref, z, f, g, n_unknowns: int):
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1, 2)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1, 2)
    pg, _ = _dev_ptr(g, "g", n_unknowns)
    _check(load_library().rw_stokeslet_rhs(ref, z.ctypes.data_as(_DP), f.ctypes.data_as(_DP), z.shape[0], pg), ctx)


class Server:
    """rw_server_*: requests (refinement + Stokeslet right-hand sides) served
    by `slots` worker threads against one resident wall."""

    def __init__(self, wall: "Wall", slots: int = 4, hbm_budget_bytes: int = 0):
        self.wall = wall
        self.h = None
        out = _P()
        rc = load_library().rw_server_create(wall.ctx.h, wall.h, wall.n_panels, slots, hbm_budget_bytes,
                                             ctypes.byref(out))
        if rc != RW_OK:
            raise RwError(rc, load_library().rw_server_error(None).decode())
        self.h = out
        self._n = {}
        wall._children.add(self)   # closed before its wall

    def _err(self, rc):
        if rc != RW_OK:
            raise RwError(rc, load_library().rw_server_error(self.h).decode())

    def submit(self, panel_ids, levels, stokeslets) -> int:
        """Queue one request; `stokeslets`: one (z, f) pair of (n_src, 2)
        arrays per right-hand side (all with the same n_src).  Returns its id."""
        ids = np.ascontiguousarray(panel_ids, dtype=np.int32)
        lev = np.ascontiguousarray(levels, dtype=np.int32)
        z = np.ascontiguousarray(np.concatenate([np.asarray(s[0], np.float64).reshape(-1, 2) for s in stokeslets]))
        f = np.ascontiguousarray(np.concatenate([np.asarray(s[1], np.float64).reshape(-1, 2) for s in stokeslets]))
        nrhs = len(stokeslets)
        n_src = z.shape[0] // nrhs
        rid = ctypes.c_int64(0)
        self._err(load_library().rw_server_submit(self.h, ids.ctypes.data_as(_I32P), lev.ctypes.data_as(_I32P),
                                                  ids.size, z.ctypes.data_as(_DP), f.ctypes.data_as(_DP), n_src,
                                                  nrhs, ctypes.byref(rid)))
        q = self.wall.n_nodes // self.wall.n_panels
        n_nodes = self.wall.n_nodes + sum(q * (2 ** int(l) - 1) for l in lev)
        self._n[rid.value] = (2 * n_nodes, nrhs)
        return rid.value

    def wait(self, rid: int, check: bool = True):
        """(tau of shape (nrhs, 2 N_n), info dict) of request rid."""
        n2, nrhs = self._n.pop(rid)
        tau = np.empty((nrhs, n2))
        inf = rw_request_info()
        rc = load_library().rw_server_wait(self.h, rid, tau.ctypes.data_as(_DP), tau.size, ctypes.byref(inf))
        info = {f: getattr(inf, f) for f, _ in rw_request_info._fields_}
        if check:
            self._err(rc)
        return tau, info

    def close(self):
        if self.h:
            load_library().rw_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- classes
class Context:
    """A device + stream + HBM budget.  Closing it first closes the walls made
    on it (and their refinements): the C ABI requires a ctx to outlive its
    walls and a wall its refinements."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, hbm_budget_bytes: int = 0, **opts):
        self.device = device
        self.h = None
        self._children = weakref.WeakSet()
        self.h = rw_ctx_create(device, stream, hbm_budget_bytes)
        if opts:
            rw_set_options(self.h, **opts)

    def set_options(self, **opts):
        rw_set_options(self.h, **opts)

    def options(self) -> dict:
        return rw_get_options(self.h)

    def bytes(self) -> int:
        return int(load_library().rw_ctx_bytes(self.h))

    def trim(self):
        rw_ctx_trim(self.h)

    def profile(self, on: bool = True):
        rw_profile_enable(self.h, on)

    def profile_reset(self):
        rw_profile_reset(self.h)

    def profile_json(self) -> dict:
        return rw_profile_json(self.h)

    def close(self):
        if self.h:
            for w in list(self._children):
                w.close()
            rw_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Wall:
    """Reference wall with its HBS compressed inverse resident in HBM."""

    def __init__(self, ctx: Context, n_panels: int, order: int = 16, leaf_nodes: int = 64,
                 id_tol: float = 1e-10, precision: int = RW_F64, a: float = 0.3, m: int = 5):
        self.ctx = ctx
        self.h = None
        self._children = weakref.WeakSet()
        if not ctx.h:
            raise RwError(RW_EINVAL, "context is closed")
        self.h = rw_wall_build(ctx.h, n_panels, order, leaf_nodes, id_tol, precision, a, m)
        ctx._children.add(self)
        self.n_nodes = n_panels * order
        self.n_panels = n_panels

    def stats(self) -> dict:
        return rw_wall_stats_get(self.ctx.h, self.h)

    def nodes(self):
        return rw_wall_nodes(self.ctx.h, self.h)

    def hbs_apply(self, b):
        import torch
        x = torch.empty_like(b)
        rw_hbs_apply(self.ctx.h, self.h, b, x, 2 * self.n_nodes)
        return x

    def refine(self, panel_ids, levels, q_tol: float = 0.0) -> "Refined":
        return Refined(self, panel_ids, levels, q_tol)

    def solve_batch(self, refs, gs, check: bool = True):
        """tau_i = A_nn(i)^{-1} g_i for refinements `refs` of this wall in one
        call (rw_solve_batch); returns ([tau_i], [info_i])."""
        import torch
        taus = [torch.empty_like(g) for g in gs]
        _, infos = rw_solve_batch(self.ctx.h, [r.h for r in refs], gs, taus, [r.n_unknowns for r in refs],
                                  check=check)
        return taus, infos

    def close(self):
        if self.h:
            for r in list(self._children):
                r.close()
            if self.ctx.h:
                rw_wall_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Refined:
    """A locally refined discretization with its Algorithm-1 factors."""

    def __init__(self, wall: Wall, panel_ids, levels, q_tol: float = 0.0):
        self.wall = wall
        self.ctx = wall.ctx
        self.h = None
        if not wall.h:
            raise RwError(RW_EINVAL, "wall is closed")
        self.h = rw_refine(self.ctx.h, wall.h, panel_ids, levels, q_tol)
        wall._children.add(self)
        self._refresh()

    def _refresh(self):
        self.info_ = rw_refined_info(self.ctx.h, self.h)
        self.n_nodes = int(self.info_["n_k"] + self.info_["n_p"])

    @property
    def n_unknowns(self) -> int:
        return 2 * self.n_nodes

    def info(self) -> dict:
        return rw_refined_info(self.ctx.h, self.h)

    def coarsen(self, panel_ids):
        rw_coarsen(self.ctx.h, self.h, panel_ids)
        self._refresh()

    def nodes(self):
        return rw_nodes(self.ctx.h, self.h)

    def stokeslet_rhs(self, z, f):
        import torch
        g = torch.empty(self.n_unknowns, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        rw_stokeslet_rhs(self.ctx.h, self.h, z, f, g, self.n_unknowns)
        return g

    def solve(self, g, check: bool = True, info: dict = None):
        import torch
        tau = torch.empty_like(g)
        rw_solve(self.ctx.h, self.h, g, tau, self.n_unknowns, check=check, info=info)
        return tau

    def residual(self, g, tau):
        import torch
        r = torch.empty_like(g)
        rw_residual(self.ctx.h, self.h, g, tau, r, self.n_unknowns)
        return r

    def close(self):
        if self.h:
            if self.wall.h and self.ctx.h:
                rw_refined_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _CachedRefined(Refined):
    """A refined handle owned by a RefCache (never freed by itself)."""

    def __init__(self, cache: "RefCache", h):
        self.wall = cache.wall
        self.ctx = cache.wall.ctx
        self.h = h
        self._refresh()

    def close(self):
        self.h = None


class RefCache:
    """rw_refcache_*: refinements reused across time steps (Sec. 5.3)."""

    def __init__(self, wall: "Wall", capacity: int = 4, margin: int = 2, q_tol: float = 0.0):
        self.wall = wall
        self.h = None
        out = _P()
        rc = load_library().rw_refcache_create(wall.h, wall.n_panels, capacity, margin, q_tol, ctypes.byref(out))
        if rc != RW_OK:
            raise RwError(rc, load_library().rw_refcache_error(None).decode())
        self.h = out
        wall._children.add(self)

    def get(self, panel_ids, levels):
        """(refined handle covering the request, hit flag)."""
        ids = np.ascontiguousarray(panel_ids, dtype=np.int32)
        lev = np.ascontiguousarray(levels, dtype=np.int32)
        out = _P()
        hit = ctypes.c_int32(0)
        rc = load_library().rw_refcache_get(self.h, ids.ctypes.data_as(_I32P), lev.ctypes.data_as(_I32P), ids.size,
                                            ctypes.byref(out), ctypes.byref(hit))
        if rc != RW_OK:
            raise RwError(rc, load_library().rw_refcache_error(self.h).decode() or
                          load_library().rw_last_error(self.wall.ctx.h).decode())
        return _CachedRefined(self, out), bool(hit.value)

    def panels(self, ref):
        n = ctypes.c_int32(0)
        _check(load_library().rw_refcache_panels(self.h, ref.h, None, None, ctypes.byref(n)), self.wall.ctx.h)
        ids = np.empty(n.value, np.int32)
        lev = np.empty(n.value, np.int32)
        _check(load_library().rw_refcache_panels(self.h, ref.h, ids.ctypes.data_as(_I32P), lev.ctypes.data_as(_I32P),
                                                 ctypes.byref(n)), self.wall.ctx.h)
        return ids, lev

    def stats(self):
        h, m, k = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
        load_library().rw_refcache_stats(self.h, ctypes.byref(h), ctypes.byref(m), ctypes.byref(k))
        return {"hits": h.value, "misses": m.value, "held": k.value}

    def close(self):
        if self.h:
            load_library().rw_refcache_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
