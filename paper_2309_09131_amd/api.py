"""PyTorch-facing wrapper of the C ABI.

PyTorch supplies device memory and the stream; every step runs in the HIP
library.  Names follow the C entry points (mttkrp_mode, mttkrp_all_modes,
remap, cp_loss_grad, cp_als_sweep, cp_als); `Plan` bundles the workspace
tensor and the plan handle, `CpLoss` exposes the sampled CP loss to autograd.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _abi

_DT = {torch.float32: _abi.F32, torch.bfloat16: _abi.BF16}


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _fdt(factors):
    dts = {f.dtype for f in factors if f is not None}
    if len(dts) != 1 or next(iter(dts)) not in _DT:
        raise ValueError("factors must all be float32 or all bfloat16")
    return _DT[next(iter(dts))]


def _ptr(t):
    if t is None:
        return 0
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return t.data_ptr()


class Plan:
    """A tensor preprocessed for all-mode MTTKRP (owns its workspace)."""

    def __init__(self, idx: torch.Tensor, vals: torch.Tensor, dims, rank: int,
                 g: int = 0, m=None, workers: int = 0, flags: int = 0):
        if idx.dtype != torch.int32 or vals.dtype != torch.float32:
            raise ValueError("idx must be int32 (N, nnz), vals float32 (nnz,)")
        self.dims = tuple(int(d) for d in dims)
        self.N = len(self.dims)
        self.nnz = int(vals.numel())
        self.rank = int(rank)
        if idx.shape != (self.N, self.nnz):
            raise ValueError(f"idx shape {tuple(idx.shape)} != {(self.N, self.nnz)}")
        self.device = vals.device
        self.opts = _abi.make_opts(g, m, workers, flags)
        nbytes = _abi.mttkrp_plan_workspace(self.N, self.dims, self.nnz, self.rank,
                                            self.opts)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8,
                                     device=self.device)
        self.handle = _abi.mttkrp_plan(self.N, self.dims, self.nnz,
                                       _ptr(idx.contiguous()), _ptr(vals.contiguous()),
                                       self.rank, self.opts, self.workspace.data_ptr(),
                                       nbytes, _stream())

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                _abi.mttkrp_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    # -- queries -------------------------------------------------------------
    @property
    def cur_mode(self):
        return _abi.mttkrp_plan_info(self.handle, _abi.INFO_CUR_MODE)

    def info(self, what, mode=0):
        return _abi.mttkrp_plan_info(self.handle, what, mode)

    def query(self, what, mode=0) -> np.ndarray:
        N = self.N
        if what == _abi.Q_LAYOUT:
            shape, dt = (self.nnz, N + 1), np.int32
        elif what == _abi.Q_PERM:
            shape, dt = (self.nnz,), np.int32
        elif what == _abi.Q_ROW_PTR:
            shape, dt = (self.dims[mode] + 1,), np.int32
        elif what == _abi.Q_SHARDS:
            shape, dt = (self.info(_abi.INFO_NSHARDS, mode), 3), np.int32
        elif what == _abi.Q_LPT:
            shape, dt = (self.info(_abi.INFO_NSUPER, mode),), np.int32
        else:
            raise ValueError(what)
        out = np.zeros(shape, dtype=dt)
        if out.size:
            _abi.mttkrp_plan_query(self.handle, what, mode, out.ctypes.data,
                                   out.nbytes, _stream())
        return out

    # -- compute -------------------------------------------------------------
    def mttkrp_mode(self, mode, factors, out=None, fuse_remap=True):
        if out is None:
            out = torch.empty((self.dims[mode], self.rank), dtype=torch.float32,
                              device=self.device)
        fac = [f if w != mode else None for w, f in enumerate(factors)]
        _abi.mttkrp_mode(self.handle, mode, [_ptr(f) for f in fac], _fdt(fac),
                         _ptr(out), fuse_remap, _stream())
        return out

    def mttkrp_all_modes(self, factors, outs=None):
        if outs is None:
            outs = [torch.empty((d, self.rank), dtype=torch.float32, device=self.device)
                    for d in self.dims]
        _abi.mttkrp_all_modes(self.handle, [_ptr(f) for f in factors], _fdt(factors),
                              [_ptr(o) for o in outs], _stream())
        return outs

    def remap(self, to_mode):
        _abi.remap(self.handle, to_mode, _stream())

    def cp_loss_grad(self, factors, loss=True, grads=True, grad_scale=None):
        dl = torch.empty((), dtype=torch.float64, device=self.device) if loss else None
        gs = [torch.empty((d, self.rank), dtype=torch.float32, device=self.device)
              for d in self.dims] if grads else None
        _abi.cp_loss_grad(self.handle, [_ptr(f) for f in factors], _fdt(factors),
                          _ptr(dl), [_ptr(g) for g in gs] if gs else None,
                          _ptr(grad_scale), _stream())
        return dl, gs

    def cp_als_sweep(self, factors, mbuf=None, lam=None, want_fit=True):
        """One CP-ALS sweep; `factors` are updated in place."""
        if mbuf is None:
            mbuf = torch.empty((max(self.dims), self.rank), dtype=torch.float32,
                               device=self.device)
        if lam is None:
            lam = torch.empty(self.rank, dtype=torch.float64, device=self.device)
        fit = torch.empty((), dtype=torch.float64, device=self.device) if want_fit else None
        _abi.cp_als_sweep(self.handle, [_ptr(f) for f in factors], _fdt(factors),
                          _ptr(mbuf), _ptr(lam), _ptr(fit), _stream())
        return lam, fit

    def cp_als_sweep_static(self, factors, lam, fit=None):
        """One CP-ALS sweep whose scratch is the library's static device
        array (no allocation in the call); `factors` are updated in place,
        `lam` (FP64, R) and `fit` (FP64 scalar or None) are written."""
        _abi.cp_als_sweep_static(self.handle, [_ptr(f) for f in factors], _fdt(factors),
                                 _ptr(lam), _ptr(fit), _stream())

    def cp_als(self, factors, max_sweeps, tol=0.0, mbuf=None, lam=None, trace=True):
        """CP-ALS until two consecutive fits differ by less than `tol` (or
        `max_sweeps` sweeps); `factors` are updated in place.  Returns
        (lambda, fits) with fits the FP64 fit after every sweep run."""
        if mbuf is None:
            mbuf = torch.empty((max(self.dims), self.rank), dtype=torch.float32,
                               device=self.device)
        if lam is None:
            lam = torch.empty(self.rank, dtype=torch.float64, device=self.device)
        tr = torch.empty(max_sweeps, dtype=torch.float64, device=self.device) if trace else None
        k, fit = _abi.cp_als(self.handle, [_ptr(f) for f in factors], _fdt(factors),
                             _ptr(mbuf), _ptr(lam), int(max_sweeps), float(tol), _ptr(tr),
                             _stream())
        return lam, (tr[:k] if trace else torch.tensor([fit], dtype=torch.float64))

    def profile(self, enable=True):
        _abi.mttkrp_profile(self.handle, enable)

    def profile_read(self, kernel=_abi.PROF_MTTKRP, mode=-1):
        """(milliseconds, launches) of `kernel` since the last read."""
        return _abi.mttkrp_profile_read(self.handle, kernel, mode)


class CpLoss(torch.autograd.Function):
    """Sampled CP loss sum_e (x_e - sum_r prod_n A_n(c_n(e), r))^2.

    forward(plan, *factors) -> float64 scalar.  When any factor needs a
    gradient, the forward evaluates loss and gradients together (the first
    residual pass of cp_loss_grad also yields the loss, so this costs N
    passes instead of 1 + N) and backward scales the kept gradients by the
    upstream gradient; otherwise the forward is the single loss pass.
    """

    @staticmethod
    def forward(ctx, plan: Plan, *factors):
        ctx.dtypes = [f.dtype for f in factors]
        if any(ctx.needs_input_grad[1:]):
            loss, grads = plan.cp_loss_grad(list(factors), loss=True, grads=True)
            ctx.grads = grads
        else:
            loss, _ = plan.cp_loss_grad(list(factors), loss=True, grads=False)
            ctx.grads = None
        return loss

    @staticmethod
    def backward(ctx, g):
        grads = ctx.grads
        ctx.grads = None
        out = [None]
        for gr in grads:
            k = len(out)
            if ctx.needs_input_grad[k]:
                # FP32 gradients (as the MTTKRP outputs), in the factor's dtype
                out.append((gr * g.detach().to(gr.dtype)).to(ctx.dtypes[k - 1]))
            else:
                out.append(None)
        return tuple(out)


def cp_loss(plan: Plan, factors):
    return CpLoss.apply(plan, *factors)
