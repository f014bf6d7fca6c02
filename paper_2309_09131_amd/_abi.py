"""ctypes binding of libmttkrp.so, one Python function per C entry point.

Argument marshalling only: every computation happens in the HIP library.
Device pointers are passed as integers (e.g. torch.Tensor.data_ptr()), the
stream as the integer handle of a hipStream_t (0 = default stream).  A
non-OK status raises RuntimeError with the library's error text.  There is
no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmttkrp.so")

MAX_MODES = 8
MAX_NNZ = (1 << 31) - (1 << 20)   # MTTKRP_MAX_NNZ
STATIC_MBUF_FLOATS = 1 << 24      # MTTKRP_STATIC_MBUF_FLOATS
OK, EINVAL, ERANGE, ENOMEM, ESTATE, EHIP = range(6)
F32, BF16 = 0, 1
NO_IMPLICIT_REMAP = 1
NATURAL_ORDER = 2
FUSED_REMAP = 4
UNPACKED_RECORDS = 8
GATHER_ONLY = 16
LOCALITY_ORDER = 32


def RESIDENT_LAYOUT(n):
    """MTTKRP_RESIDENT_LAYOUT(n): keep the layout of mode n resident."""
    return 1 << (16 + n)
PROF_MTTKRP, PROF_REMAP, PROF_RESID, PROF_LOSS = 0, 1, 2, 3
Q_LAYOUT, Q_PERM, Q_ROW_PTR, Q_SHARDS, Q_LPT = range(5)
INFO_CUR_MODE, INFO_NSHARDS, INFO_NSUPER = 0, 1, 2
INFO_NSPLIT, INFO_G, INFO_M, INFO_RIDGE = 4, 5, 6, 7
INFO_RECORD_BYTES = 8

SYMBOLS = ["mttkrp_plan_workspace", "mttkrp_plan", "mttkrp_mode",
           "mttkrp_all_modes", "remap", "cp_loss_grad", "cp_als_sweep",
           "cp_als_sweep_static", "cp_als",
           "mttkrp_plan_query", "mttkrp_plan_info", "mttkrp_profile",
           "mttkrp_profile_read", "mttkrp_plan_destroy", "mttkrp_status_str",
           "mttkrp_last_error"]


class Opts(ctypes.Structure):
    _fields_ = [("g", ctypes.c_int32), ("m", ctypes.c_int32 * MAX_MODES),
                ("workers", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class MttkrpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built; run __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname as the system's;
    # whichever is loaded first serves the whole process, so torch is loaded
    # before the library resolves its HIP dependency
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "mttkrp_plan_workspace": [_int, _vp, _i64, _int, _vp, _vp],
        "mttkrp_plan": [_int, _vp, _i64, _vp, _vp, _int, _vp, _vp, ctypes.c_size_t,
                        _vp, _vp],
        "mttkrp_mode": [_vp, _int, _vp, _int, _vp, _int, _vp],
        "mttkrp_all_modes": [_vp, _vp, _int, _vp, _vp],
        "remap": [_vp, _int, _vp],
        "cp_loss_grad": [_vp, _vp, _int, _vp, _vp, _vp, _vp],
        "cp_als_sweep": [_vp, _vp, _int, _vp, _vp, _vp, _vp],
        "cp_als_sweep_static": [_vp, _vp, _int, _vp, _vp, _vp],
        "cp_als": [_vp, _vp, _int, _vp, _vp, _int, ctypes.c_double, _vp,
                   ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double), _vp],
        "mttkrp_plan_query": [_vp, _int, _int, _vp, ctypes.c_size_t, _vp],
        "mttkrp_plan_info": [_vp, _int, _int, ctypes.POINTER(_i64)],
        "mttkrp_profile": [_vp, _int],
        "mttkrp_profile_read": [_vp, _int, _int, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(_i64)],
        "mttkrp_plan_destroy": [_vp],
        "mttkrp_status_str": [_int],
        "mttkrp_last_error": [_vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("mttkrp_status_str",
                                                 "mttkrp_last_error") else _int
    _lib = lib
    return lib


def _check(st, plan=None):
    if st != OK:
        lib = load()
        msg = lib.mttkrp_last_error(plan).decode()
        raise MttkrpError(st, f"{lib.mttkrp_status_str(st).decode()}: {msg}")


def _dims(dims):
    return (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])


def _ptrs(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])


def make_opts(g=0, m=None, workers=0, flags=0):
    o = Opts()
    o.g = int(g)
    for n, v in enumerate(m or []):
        o.m[n] = int(v)
    o.workers = int(workers)
    o.flags = int(flags)
    return o


def mttkrp_plan_workspace(nmodes, dims, nnz, rank, opts=None):
    lib = load()
    out = ctypes.c_size_t(0)
    _check(lib.mttkrp_plan_workspace(nmodes, _dims(dims), nnz, rank,
                                     ctypes.byref(opts) if opts else None,
                                     ctypes.byref(out)))
    return out.value


def mttkrp_plan(nmodes, dims, nnz, d_idx, d_vals, rank, opts, d_ws, ws_bytes,
                stream=0):
    lib = load()
    h = ctypes.c_void_p(None)
    _check(lib.mttkrp_plan(nmodes, _dims(dims), nnz, d_idx, d_vals, rank,
                           ctypes.byref(opts) if opts else None, d_ws, ws_bytes,
                           stream or None, ctypes.byref(h)))
    return h.value


def mttkrp_mode(plan, mode, d_factors, fdt, d_out, fuse_remap, stream=0):
    lib = load()
    _check(lib.mttkrp_mode(plan, mode, _ptrs(d_factors), fdt, d_out,
                           1 if fuse_remap else 0, stream or None), plan)


def mttkrp_all_modes(plan, d_factors, fdt, d_outs, stream=0):
    lib = load()
    _check(lib.mttkrp_all_modes(plan, _ptrs(d_factors), fdt, _ptrs(d_outs),
                                stream or None), plan)


def remap(plan, to_mode, stream=0):
    lib = load()
    _check(lib.remap(plan, to_mode, stream or None), plan)


def cp_loss_grad(plan, d_factors, fdt, d_loss, d_grads, d_grad_scale, stream=0):
    lib = load()
    _check(lib.cp_loss_grad(plan, _ptrs(d_factors), fdt, d_loss or None,
                            _ptrs(d_grads) if d_grads else None,
                            d_grad_scale or None, stream or None), plan)


def cp_als_sweep(plan, d_factors, fdt, d_mbuf, d_lambda, d_fit, stream=0):
    lib = load()
    _check(lib.cp_als_sweep(plan, _ptrs(d_factors), fdt, d_mbuf, d_lambda,
                            d_fit or None, stream or None), plan)


def cp_als_sweep_static(plan, d_factors, fdt, d_lambda, d_fit, stream=0):
    lib = load()
    _check(lib.cp_als_sweep_static(plan, _ptrs(d_factors), fdt, d_lambda, d_fit or None,
                                   stream or None), plan)


def cp_als(plan, d_factors, fdt, d_mbuf, d_lambda, max_sweeps, tol, d_fit_trace=0, stream=0):
    """Returns (sweeps run, last fit)."""
    lib = load()
    sweeps = _int(0)
    fit = ctypes.c_double(0.0)
    _check(lib.cp_als(plan, _ptrs(d_factors), fdt, d_mbuf, d_lambda, max_sweeps, tol,
                      d_fit_trace or None, ctypes.byref(sweeps), ctypes.byref(fit),
                      stream or None), plan)
    return sweeps.value, fit.value


def mttkrp_plan_query(plan, what, mode, dst, nbytes, stream=0):
    lib = load()
    _check(lib.mttkrp_plan_query(plan, what, mode, dst, nbytes, stream or None),
           plan)


def mttkrp_plan_info(plan, what, mode=0):
    lib = load()
    v = ctypes.c_int64(0)
    _check(lib.mttkrp_plan_info(plan, what, mode, ctypes.byref(v)), plan)
    return v.value


def mttkrp_profile(plan, enable):
    lib = load()
    _check(lib.mttkrp_profile(plan, 1 if enable else 0), plan)


def mttkrp_profile_read(plan, kernel=0, mode=-1):
    lib = load()
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib.mttkrp_profile_read(plan, kernel, mode, ctypes.byref(ms),
                                   ctypes.byref(cnt)), plan)
    return ms.value, cnt.value


def mttkrp_plan_destroy(plan):
    lib = load()
    _check(lib.mttkrp_plan_destroy(plan))


def mttkrp_status_str(st):
    return load().mttkrp_status_str(st).decode()


def mttkrp_last_error(plan=None):
    return load().mttkrp_last_error(plan).decode()
