"""ctypes binding of the C ABI in include/lqcd.h (argument marshalling only).

Every call forwards device pointers (``torch.Tensor.data_ptr()``), sizes and
a HIP stream handle to ``lib/liblqcd.so``; all work runs in the library's
HIP kernels.  Importing this module fails loudly if the library has not been
built (``python -m paper_1411_5219_amd.build``).
"""

from __future__ import annotations

import ctypes
import math
import os

# LQCD_LIBRARY selects another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("LQCD_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib",
                                                          "liblqcd.so")

OK, EINVAL, EUNSUPPORTED, ENOCONV, EBREAKDOWN, ENONFINITE, EHIP = 0, -1, -2, -3, -4, -5, -6
PREC_64, PREC_32, PREC_16 = 64, 32, 16
RECON_18, RECON_12 = 18, 12
OP_HOP, OP_SCHUR, OP_NORMAL = 0, 1, 2
FIELD_SPINOR_PARITY, FIELD_SPINOR_FULL, FIELD_GAUGE, FIELD_COLOUR_PARITY, FIELD_COLOUR_FULL = 0, 1, 2, 3, 4

ERROR_NAMES = {OK: "OK", EINVAL: "EINVAL", EUNSUPPORTED: "EUNSUPPORTED", ENOCONV: "ENOCONV",
               EBREAKDOWN: "EBREAKDOWN", ENONFINITE: "ENONFINITE", EHIP: "EHIP"}

# Every symbol the header declares.
SYMBOLS = ["lqcd_last_error", "lqcd_version", "lqcd_device_memory", "lqcd_field_bytes", "lqcd_workspace_bytes", "lqcd_set_launch",
           "lqcd_get_launch", "lqcd_autotune_dslash", "lqcd_pack_gauge",
           "lqcd_pack_spinor", "lqcd_unpack_spinor", "dslash_apply", "dslash_eo_apply", "cg_solve",
           "bicgstab_solve", "lqcd_workspace_bytes_batch", "cg_solve_batch", "lqcd_pack_colour",
           "lqcd_unpack_colour", "stag_apply", "stag_eo_apply", "lqcd_workspace_bytes_stag", "stag_cg_solve",
           "stag_multishift_solve", "lqcd_autotune_stag", "lqcd_autotune_dslash_rhs", "lqcd_gamma5", "tm_force",
           "dslash_eo_apply_noalloc", "lqcd_autotune_batch", "lqcd_tune_cache_load", "lqcd_tune_cache_save",
           "lqcd_tune_cache_clear", "lqcd_tune_cache_put", "lqcd_tune_cache_get"]


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("theta", ctypes.c_double * 4)]


class Op(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("mu", ctypes.c_double), ("prec", ctypes.c_int32),
                ("recon", ctypes.c_int32)]


class StagOp(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("prec", ctypes.c_int32), ("recon", ctypes.c_int32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int32), ("eo", ctypes.c_int32),
                ("inner_prec", ctypes.c_int32), ("inner_recon", ctypes.c_int32), ("nrhs", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("delta_reliable", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("stag_window", ctypes.c_int32), ("tol_inner", ctypes.c_double),
                ("max_stagnations", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("bicgstab_ell", ctypes.c_int32)]


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("swizzle", ctypes.c_int32), ("order", ctypes.c_int32),
                ("rhs_tile", ctypes.c_int32), ("rhs_group", ctypes.c_int32), ("ygroup", ctypes.c_int32),
                ("rhs_lanes", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


KERNEL_DSLASH, KERNEL_BLAS, KERNEL_STAG, KERNEL_DSLASH_RHS = 0, 1, 2, 3


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("true_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("hops_outer", ctypes.c_double), ("hops_inner", ctypes.c_double),
                ("outer_iters", ctypes.c_int32), ("stagnations", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("persistent_launches", ctypes.c_int32), ("eo_resid", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LqcdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is missing: build it with "
                          "`python -m paper_1411_5219_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, szp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)
    G, O, P, I = ctypes.POINTER(Geom), ctypes.POINTER(Op), ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo)
    SO = ctypes.POINTER(StagOp)
    sig = {
        "lqcd_last_error": ([], ctypes.c_char_p),
        "lqcd_version": ([], ctypes.c_char_p),
        "lqcd_device_memory": ([i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], ctypes.c_int),
        "lqcd_field_bytes": ([G, i32, i32, i32, szp], ctypes.c_int),
        "lqcd_workspace_bytes": ([G, O, P, szp], ctypes.c_int),
        "lqcd_set_launch": ([i32, i32, ctypes.POINTER(Launch)], ctypes.c_int),
        "lqcd_get_launch": ([i32, i32, ctypes.POINTER(Launch)], ctypes.c_int),
        "lqcd_autotune_dslash": ([G, O, vp, vp, vp, i32, vp, ctypes.POINTER(Launch), ctypes.POINTER(ctypes.c_double)],
                                 ctypes.c_int),
        "lqcd_pack_gauge": ([G, i32, i32, vp, vp, vp], ctypes.c_int),
        "lqcd_pack_spinor": ([G, i32, i32, vp, vp, vp], ctypes.c_int),
        "lqcd_unpack_spinor": ([G, i32, i32, vp, vp, vp], ctypes.c_int),
        "dslash_apply": ([G, O, vp, vp, vp, i32, i32, vp, vp], ctypes.c_int),
        "dslash_eo_apply": ([G, O, vp, vp, vp, i32, i32, i32, i32, vp, vp], ctypes.c_int),
        "dslash_eo_apply_noalloc": ([G, O, vp, vp, vp, i32, i32, i32, i32, vp], ctypes.c_int),
        "cg_solve": ([G, O, vp, vp, vp, P, I, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "bicgstab_solve": ([G, O, vp, vp, vp, P, I, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "lqcd_workspace_bytes_batch": ([i32, G, O, P, szp], ctypes.c_int),
        "cg_solve_batch": ([i32, G, O, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), P, I, vp,
                            ctypes.c_size_t, vp], ctypes.c_int),
        "lqcd_autotune_batch": ([i32, G, O, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), P, vp,
                                 ctypes.c_size_t, i32, vp, ctypes.POINTER(Launch), ctypes.POINTER(ctypes.c_double)],
                                ctypes.c_int),
        "lqcd_tune_cache_load": ([ctypes.c_char_p], ctypes.c_int),
        "lqcd_tune_cache_save": ([ctypes.c_char_p], ctypes.c_int),
        "lqcd_tune_cache_clear": ([], ctypes.c_int),
        "lqcd_tune_cache_put": ([i32, i32, i32, G, i32, ctypes.POINTER(Launch), ctypes.c_double], ctypes.c_int),
        "lqcd_tune_cache_get": ([i32, i32, i32, G, i32, ctypes.POINTER(Launch), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(i32)], ctypes.c_int),
        "lqcd_pack_colour": ([G, i32, i32, vp, vp, vp], ctypes.c_int),
        "lqcd_unpack_colour": ([G, i32, i32, vp, vp, vp], ctypes.c_int),
        "stag_apply": ([G, SO, vp, vp, vp, i32, i32, vp], ctypes.c_int),
        "stag_eo_apply": ([G, SO, vp, vp, vp, i32, i32, i32, vp, vp], ctypes.c_int),
        "lqcd_workspace_bytes_stag": ([G, SO, i32, szp], ctypes.c_int),
        "lqcd_autotune_stag": ([G, SO, vp, vp, vp, i32, vp, ctypes.POINTER(Launch), ctypes.POINTER(ctypes.c_double)],
                               ctypes.c_int),
        "lqcd_autotune_dslash_rhs": ([G, O, vp, vp, vp, i32, i32, vp, ctypes.POINTER(Launch),
                                      ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "lqcd_gamma5": ([G, i32, vp, vp, vp], ctypes.c_int),
        "tm_force": ([G, O, vp, vp, vp, vp, ctypes.c_double, i32, vp], ctypes.c_int),
        "stag_cg_solve": ([G, SO, vp, vp, vp, P, I, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "stag_multishift_solve": ([G, SO, vp, vp, vp, ctypes.POINTER(ctypes.c_double), i32, P, I, vp,
                                   ctypes.c_size_t, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc):
    if rc != OK:
        raise LqcdError(rc, lqcd_last_error())
    return rc


def geom(L, theta=(0.0, 0.0, 0.0, math.pi)) -> Geom:
    g = Geom()
    for m in range(4):
        g.L[m] = int(L[m])
        g.theta[m] = float(theta[m])
    return g


def op(kappa, mu=0.0, prec=64, recon=18) -> Op:
    return Op(float(kappa), float(mu), int(prec), int(recon))


def solve_params(tol=1e-10, maxiter=10000, eo=1, inner_prec=64, inner_recon=12, nrhs=1, use_graph=0,
                 delta_reliable=0.1, check_every=8, stag_window=0, tol_inner=0.0, max_stagnations=0,
                 persistent=0, bicgstab_ell=0) -> SolveParams:
    return SolveParams(float(tol), int(maxiter), int(eo), int(inner_prec), int(inner_recon), int(nrhs),
                       int(use_graph), float(delta_reliable), int(check_every), int(stag_window), float(tol_inner),
                       int(max_stagnations), int(persistent), int(bicgstab_ell))


def lqcd_last_error() -> str:
    return _lib.lqcd_last_error().decode()


def lqcd_version() -> str:
    return _lib.lqcd_version().decode()


def lqcd_field_bytes(g, kind, prec, recon=18) -> int:
    n = ctypes.c_size_t()
    _check(_lib.lqcd_field_bytes(ctypes.byref(g), kind, prec, recon, ctypes.byref(n)))
    return n.value


def lqcd_workspace_bytes(g, o, params=None) -> int:
    n = ctypes.c_size_t()
    p = ctypes.byref(params) if params is not None else None
    _check(_lib.lqcd_workspace_bytes(ctypes.byref(g), ctypes.byref(o), p, ctypes.byref(n)))
    return n.value


def lqcd_set_launch(kernel, prec, block, swizzle=1, order=0, rhs_tile=1, rhs_group=0, ygroup=1, rhs_lanes=1):
    cfg = Launch(int(block), int(swizzle), int(order), int(rhs_tile), int(rhs_group), int(ygroup), int(rhs_lanes))
    return _check(_lib.lqcd_set_launch(int(kernel), int(prec), ctypes.byref(cfg)))


def lqcd_get_launch(kernel, prec):
    l = Launch()
    _check(_lib.lqcd_get_launch(int(kernel), int(prec), ctypes.byref(l)))
    return l.as_dict()


def lqcd_autotune_dslash(g, o, U, inp, out, reps=10, stream=None):
    """Returns ({block, swizzle, order}, mean launch microseconds) and installs the winner."""
    best = Launch()
    us = ctypes.c_double()
    _check(_lib.lqcd_autotune_dslash(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(inp), _ptr(out), int(reps),
                                     _stream(stream), ctypes.byref(best), ctypes.byref(us)))
    return (best.as_dict(), us.value)


def lqcd_pack_gauge(g, prec, recon, U_canonical, U_out, stream=None):
    return _check(_lib.lqcd_pack_gauge(ctypes.byref(g), prec, recon, _ptr(U_canonical), _ptr(U_out),
                                       _stream(stream)))


def lqcd_pack_spinor(g, prec, nrhs, psi_canonical, out, stream=None):
    return _check(_lib.lqcd_pack_spinor(ctypes.byref(g), prec, nrhs, _ptr(psi_canonical), _ptr(out),
                                        _stream(stream)))


def lqcd_unpack_spinor(g, prec, nrhs, inp, psi_canonical, stream=None):
    return _check(_lib.lqcd_unpack_spinor(ctypes.byref(g), prec, nrhs, _ptr(inp), _ptr(psi_canonical),
                                          _stream(stream)))


def dslash_apply(g, o, U, inp, out, dagger=0, nrhs=1, ws=None, stream=None):
    return _check(_lib.dslash_apply(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(inp), _ptr(out), int(dagger),
                                    int(nrhs), _ptr(ws), _stream(stream)))


def dslash_eo_apply(g, o, U, inp, out, out_parity, op_kind=OP_HOP, dagger=0, nrhs=1, ws=None, stream=None):
    return _check(_lib.dslash_eo_apply(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(inp), _ptr(out),
                                       int(out_parity), int(op_kind), int(dagger), int(nrhs), _ptr(ws),
                                       _stream(stream)))


def dslash_eo_apply_noalloc(g, o, U, inp, out, out_parity, op_kind=OP_HOP, dagger=0, nrhs=1, stream=None):
    """dslash_eo_apply without a workspace (the library's own device array holds the temporary)."""
    return _check(_lib.dslash_eo_apply_noalloc(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(inp), _ptr(out),
                                               int(out_parity), int(op_kind), int(dagger), int(nrhs),
                                               _stream(stream)))


def _solve(fn, g, o, U, b, x, params, ws, stream):
    infos = (SolveInfo * params.nrhs)()
    nbytes = ws.numel() * ws.element_size() if hasattr(ws, "numel") else 0
    rc = fn(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(b), _ptr(x), ctypes.byref(params), infos, _ptr(ws),
            nbytes, _stream(stream))
    if rc in (EINVAL, EUNSUPPORTED, EHIP):
        raise LqcdError(rc, lqcd_last_error())
    return rc, [i.as_dict() for i in infos]


def cg_solve(g, o, U, b, x, params, ws, stream=None):
    """Returns (status, [info per right-hand side]); raises on EINVAL / EUNSUPPORTED / EHIP."""
    return _solve(_lib.cg_solve, g, o, U, b, x, params, ws, stream)


def bicgstab_solve(g, o, U, b, x, params, ws, stream=None):
    return _solve(_lib.bicgstab_solve, g, o, U, b, x, params, ws, stream)


def lqcd_workspace_bytes_batch(geoms, ops, params) -> int:
    n = len(geoms)
    G = (Geom * n)(*geoms)
    O = (Op * n)(*ops)
    out = ctypes.c_size_t()
    _check(_lib.lqcd_workspace_bytes_batch(n, G, O, ctypes.byref(params), ctypes.byref(out)))
    return out.value


def cg_solve_batch(geoms, ops, Us, bs, xs, params, ws, stream=None):
    """Solve len(geoms) systems together.  Returns (status, [[info per rhs] per system])."""
    n = len(geoms)
    G = (Geom * n)(*geoms)
    O = (Op * n)(*ops)
    vp = ctypes.c_void_p
    Up = (vp * n)(*[_ptr(u) for u in Us])
    Bp = (vp * n)(*[_ptr(v) for v in bs])
    Xp = (vp * n)(*[_ptr(v) for v in xs])
    infos = (SolveInfo * (n * params.nrhs))()
    nbytes = ws.numel() * ws.element_size() if hasattr(ws, "numel") else 0
    rc = _lib.cg_solve_batch(n, G, O, Up, Bp, Xp, ctypes.byref(params), infos, _ptr(ws), nbytes, _stream(stream))
    if rc in (EINVAL, EUNSUPPORTED, EHIP):
        raise LqcdError(rc, lqcd_last_error())
    flat = [i.as_dict() for i in infos]
    return rc, [flat[s * params.nrhs:(s + 1) * params.nrhs] for s in range(n)]


def lqcd_tune_cache_load(path):
    _check(_lib.lqcd_tune_cache_load(os.fsencode(path)))


def lqcd_tune_cache_save(path):
    _check(_lib.lqcd_tune_cache_save(os.fsencode(path)))


def lqcd_tune_cache_clear():
    _check(_lib.lqcd_tune_cache_clear())


def lqcd_tune_cache_put(kernel, prec, recon, g, nrhs, launch, us=0.0):
    """Add or replace the cached shape for this key; launch is a dict as lqcd_get_launch returns."""
    cfg = Launch(**{k: int(launch[k]) for k, _ in Launch._fields_})
    _check(_lib.lqcd_tune_cache_put(int(kernel), int(prec), int(recon), ctypes.byref(g), int(nrhs),
                                    ctypes.byref(cfg), float(us)))


def lqcd_tune_cache_get(kernel, prec, recon, g, nrhs):
    """(launch dict a launch on this key uses, cached microseconds, found in the cache)."""
    cfg = Launch()
    us = ctypes.c_double()
    found = ctypes.c_int32()
    _check(_lib.lqcd_tune_cache_get(int(kernel), int(prec), int(recon), ctypes.byref(g), int(nrhs),
                                    ctypes.byref(cfg), ctypes.byref(us), ctypes.byref(found)))
    return cfg.as_dict(), us.value, bool(found.value)


def lqcd_autotune_batch(geoms, ops, Us, bs, xs, params, ws, iters=8, stream=None):
    """Time the batch's CGNR iteration per inner-hop launch shape and keep the
    fastest; returns (launch dict, microseconds per iteration).  xs and ws are
    overwritten."""
    n = len(geoms)
    G = (Geom * n)(*geoms)
    O = (Op * n)(*ops)
    vp = ctypes.c_void_p
    Up = (vp * n)(*[_ptr(u) for u in Us])
    Bp = (vp * n)(*[_ptr(v) for v in bs])
    Xp = (vp * n)(*[_ptr(v) for v in xs])
    best = Launch()
    us = ctypes.c_double()
    nbytes = ws.numel() * ws.element_size() if hasattr(ws, "numel") else 0
    _check(_lib.lqcd_autotune_batch(n, G, O, Up, Bp, Xp, ctypes.byref(params), _ptr(ws), nbytes, int(iters),
                                    _stream(stream), ctypes.byref(best), ctypes.byref(us)))
    return best.as_dict(), us.value


# ---------------------------------------------------------------------------
# Staggered fermions


def stag_op(mass, prec=64, recon=18) -> StagOp:
    return StagOp(float(mass), int(prec), int(recon))


def lqcd_pack_colour(g, prec, nrhs, chi_canonical, out, stream=None):
    return _check(_lib.lqcd_pack_colour(ctypes.byref(g), int(prec), int(nrhs), _ptr(chi_canonical), _ptr(out),
                                        _stream(stream)))


def lqcd_unpack_colour(g, prec, nrhs, inp, chi_canonical, stream=None):
    return _check(_lib.lqcd_unpack_colour(ctypes.byref(g), int(prec), int(nrhs), _ptr(inp), _ptr(chi_canonical),
                                          _stream(stream)))


def stag_apply(g, o, U, inp, out, dagger=0, nrhs=1, stream=None):
    return _check(_lib.stag_apply(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(inp), _ptr(out), int(dagger),
                                  int(nrhs), _stream(stream)))


def stag_eo_apply(g, o, U, inp, out, out_parity, op_kind=OP_HOP, nrhs=1, ws=None, stream=None):
    return _check(_lib.stag_eo_apply(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(inp), _ptr(out),
                                     int(out_parity), int(op_kind), int(nrhs), _ptr(ws), _stream(stream)))


def lqcd_workspace_bytes_stag(g, o, nshift=0) -> int:
    n = ctypes.c_size_t()
    _check(_lib.lqcd_workspace_bytes_stag(ctypes.byref(g), ctypes.byref(o), int(nshift), ctypes.byref(n)))
    return n.value


def stag_cg_solve(g, o, U, b, x, params, ws, stream=None):
    """Returns (status, info); raises on EINVAL / EUNSUPPORTED / EHIP."""
    info = SolveInfo()
    nbytes = ws.numel() * ws.element_size() if hasattr(ws, "numel") else 0
    rc = _lib.stag_cg_solve(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(b), _ptr(x), ctypes.byref(params),
                            ctypes.byref(info), _ptr(ws), nbytes, _stream(stream))
    if rc in (EINVAL, EUNSUPPORTED, EHIP):
        raise LqcdError(rc, lqcd_last_error())
    return rc, info.as_dict()


def stag_multishift_solve(g, o, U, b, x, shifts, params, ws, stream=None):
    """Returns (status, [info per shift]); raises on EINVAL / EUNSUPPORTED / EHIP."""
    n = len(shifts)
    sh = (ctypes.c_double * n)(*[float(v) for v in shifts])
    infos = (SolveInfo * n)()
    nbytes = ws.numel() * ws.element_size() if hasattr(ws, "numel") else 0
    rc = _lib.stag_multishift_solve(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(b), _ptr(x), sh, n,
                                    ctypes.byref(params), infos, _ptr(ws), nbytes, _stream(stream))
    if rc in (EINVAL, EUNSUPPORTED, EHIP):
        raise LqcdError(rc, lqcd_last_error())
    return rc, [i.as_dict() for i in infos]


def lqcd_autotune_stag(g, o, U, inp, out, reps=10, stream=None):
    best = Launch()
    us = ctypes.c_double()
    _check(_lib.lqcd_autotune_stag(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(inp), _ptr(out), int(reps),
                                   _stream(stream), ctypes.byref(best), ctypes.byref(us)))
    return (best.as_dict(), us.value)


def lqcd_autotune_dslash_rhs(g, o, U, inp, out, nrhs, reps=10, stream=None):
    """Tunes the launch shape of hops on nrhs stacked fields (block request, tile, group) and installs it
    as KERNEL_DSLASH_RHS; returns (launch, us per launch)."""
    best = Launch()
    us = ctypes.c_double()
    _check(_lib.lqcd_autotune_dslash_rhs(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(inp), _ptr(out), int(nrhs),
                                         int(reps), _stream(stream), ctypes.byref(best), ctypes.byref(us)))
    return (best.as_dict(), us.value)


# ---------------------------------------------------------------------------
# Twisted-mass pseudo-fermion force


def lqcd_device_memory(device=0):
    """(memory clock in kHz, bus width in bits) as the HIP runtime reports them."""
    c, w = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.lqcd_device_memory(int(device), ctypes.byref(c), ctypes.byref(w)))
    return c.value, w.value


def lqcd_gamma5(g, inp, out, nrhs=1, stream=None):
    return _check(_lib.lqcd_gamma5(ctypes.byref(g), int(nrhs), _ptr(inp), _ptr(out), _stream(stream)))


def tm_force(g, o, U, X, Wf, F, scale=1.0, accumulate=0, stream=None):
    return _check(_lib.tm_force(ctypes.byref(g), ctypes.byref(o), _ptr(U), _ptr(X), _ptr(Wf), _ptr(F), float(scale),
                                int(accumulate), _stream(stream)))
