"""FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's cpu_baseline leg may import
this package.  The product path never calls it.  It wraps liboracle.so
(plain single-threaded C, built from oracle.c) with numpy marshalling; it
shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile oracle.c (gcc -O2, no fast-math, no OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, os.path.join(_HERE, "oracle.c"),
                               "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = ctypes.CDLL(_SO)
        _lib.oracle_cp_loss_grad.restype = ctypes.c_int
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int64))


def _idx(idx):
    return np.ascontiguousarray(np.asarray(idx, dtype=np.int32))


def _vals(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64))


def _facs(factors):
    fs = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in factors]
    arr = (ctypes.c_void_p * len(fs))(*[f.ctypes.data for f in fs])
    return fs, arr


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def mttkrp(dims, idx, vals, factors, mode, with_abs=False):
    lib = _load()
    dims, idx, vals = _dims(dims), _idx(idx), _vals(vals)
    N, nnz = idx.shape
    fs, arr = _facs(factors)
    R = fs[0].shape[1]
    out = np.zeros((dims[mode], R))
    oabs = np.zeros((dims[mode], R)) if with_abs else None
    rc = lib.oracle_mttkrp(ctypes.c_int(N), _p(dims), ctypes.c_int64(nnz),
                           _p(idx), _p(vals), ctypes.c_int(R), arr,
                           ctypes.c_int(mode), _p(out),
                           _p(oabs) if with_abs else None)
    _check(rc, "mttkrp")
    return (out, oabs) if with_abs else out


def mttkrp_rows(dims, idx, vals, factors, mode, rows):
    lib = _load()
    dims, idx, vals = _dims(dims), _idx(idx), _vals(vals)
    N, nnz = idx.shape
    fs, arr = _facs(factors)
    R = fs[0].shape[1]
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    out = np.zeros((rows.shape[0], R))
    oabs = np.zeros((rows.shape[0], R))
    rc = lib.oracle_mttkrp_rows(ctypes.c_int(N), _p(dims), ctypes.c_int64(nnz),
                                _p(idx), _p(vals), ctypes.c_int(R), arr,
                                ctypes.c_int(mode), ctypes.c_int64(rows.shape[0]),
                                _p(rows), _p(out), _p(oabs))
    _check(rc, "mttkrp_rows")
    return out, oabs


def canonical_order(idx):
    lib = _load()
    idx = _idx(idx)
    N, nnz = idx.shape
    order = np.empty(nnz, dtype=np.int64)
    _check(lib.oracle_canonical_order(ctypes.c_int(N), ctypes.c_int64(nnz),
                                      _p(idx), _p(order)), "canonical_order")
    return order


def remap_replay(dims, idx, l0=None):
    """Returns (layouts (N+1, nnz), perm (N, nnz), row_ptrs list)."""
    lib = _load()
    dims, idx = _dims(dims), _idx(idx)
    N, nnz = idx.shape
    if l0 is None:
        l0 = canonical_order(idx)
    l0 = np.ascontiguousarray(l0, dtype=np.int64)
    layouts = np.empty((N + 1, nnz), dtype=np.int64)
    perm = np.empty((N, nnz), dtype=np.int64)
    rp = np.empty(int(np.sum(dims + 1)), dtype=np.int64)
    _check(lib.oracle_remap_replay(ctypes.c_int(N), _p(dims), ctypes.c_int64(nnz),
                                   _p(idx), _p(l0), _p(layouts), _p(perm),
                                   _p(rp)), "remap_replay")
    row_ptrs, off = [], 0
    for n in range(N):
        row_ptrs.append(rp[off:off + dims[n] + 1].copy())
        off += dims[n] + 1
    return layouts, perm, row_ptrs


def locality_layouts(dims, idx):
    """Layouts under the locality order (rows contiguous; inside a row the
    Morton code of the two leading inputs, then the other inputs, then input
    position) and their remap targets.  Returns (layouts (N+1, nnz), perm
    (N, nnz))."""
    lib = _load()
    dims, idx = _dims(dims), _idx(idx)
    N, nnz = idx.shape
    layouts = np.empty((N + 1, nnz), dtype=np.int64)
    perm = np.empty((N, nnz), dtype=np.int64)
    _check(lib.oracle_locality_layouts(ctypes.c_int(N), _p(dims), ctypes.c_int64(nnz),
                                       _p(idx), _p(layouts), _p(perm)), "locality_layouts")
    return layouts, perm


def shards(I, row_ptr, m, g):
    """Super-shard and shard tables for one mode."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    k = (I + m - 1) // m
    nnz = int(row_ptr[-1])
    bound = (nnz + g - 1) // g + k + 1
    ss_nnz = np.zeros(k, np.int64)
    ss_sh = np.zeros(k, np.int64)
    st = np.zeros(bound, np.int64)
    ln = np.zeros(bound, np.int64)
    ss = np.zeros(bound, np.int64)
    ns = ctypes.c_int64(0)
    _check(lib.oracle_shards(ctypes.c_int64(I), _p(row_ptr), ctypes.c_int64(m),
                             ctypes.c_int64(g), _p(ss_nnz), _p(ss_sh), _p(st),
                             _p(ln), _p(ss), ctypes.byref(ns)), "shards")
    s = ns.value
    return dict(ss_nnz=ss_nnz, ss_shards=ss_sh, start=st[:s], len=ln[:s],
                ss=ss[:s])


def lpt(weights, nu):
    lib = _load()
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.int64))
    bins = np.zeros(w.shape[0], np.int32)
    load = np.zeros(nu, np.int64)
    _check(lib.oracle_lpt(ctypes.c_int64(w.shape[0]), _p(w), ctypes.c_int(nu),
                          _p(bins), _p(load)), "lpt")
    return bins, load


def cp_als_sweep(dims, idx, vals, factors):
    """One Gauss-Seidel CP-ALS sweep.  Returns (factors, lambda, fit,
    ridge_count, per-mode residual^2)."""
    lib = _load()
    dims, idx, vals = _dims(dims), _idx(idx), _vals(vals)
    N, nnz = idx.shape
    fs, arr = _facs([np.array(f, dtype=np.float64, copy=True) for f in factors])
    R = fs[0].shape[1]
    lam = np.zeros(R)
    fit = ctypes.c_double(0.0)
    ridge = ctypes.c_int(0)
    res = np.zeros(N)
    _check(lib.oracle_cp_als_sweep(ctypes.c_int(N), _p(dims), ctypes.c_int64(nnz),
                                   _p(idx), _p(vals), ctypes.c_int(R), arr,
                                   _p(lam), ctypes.byref(fit),
                                   ctypes.byref(ridge), _p(res)), "cp_als_sweep")
    return fs, lam, fit.value, ridge.value, res


def cp_loss_grad(dims, idx, vals, factors, want_grad=True):
    lib = _load()
    dims, idx, vals = _dims(dims), _idx(idx), _vals(vals)
    N, nnz = idx.shape
    fs, arr = _facs(factors)
    R = fs[0].shape[1]
    loss = ctypes.c_double(0.0)
    grads = [np.zeros((dims[k], R)) for k in range(N)] if want_grad else None
    garr = (ctypes.c_void_p * N)(*[g.ctypes.data for g in grads]) \
        if want_grad else None
    _check(lib.oracle_cp_loss_grad(ctypes.c_int(N), _p(dims), ctypes.c_int64(nnz),
                                   _p(idx), _p(vals), ctypes.c_int(R), arr,
                                   ctypes.byref(loss), garr), "cp_loss_grad")
    return (loss.value, grads) if want_grad else loss.value
