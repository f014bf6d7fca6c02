"""Shared helpers of the GPU parity tests (oracle comparison, tolerances)."""
import sys

import numpy as np
import torch

import oracle
from paper_2309_09131_amd import _abi
from paper_2309_09131_amd.api import Plan

FP32_TOL = 1e-5     # relative, normwise and |.|-scaled elementwise
BF16_TOL = 2e-2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch.device("cuda:0")


def to_dev(t, dtype=torch.float32):
    d = dev()
    idx = torch.from_numpy(np.ascontiguousarray(t.idx)).to(d)
    vals = torch.from_numpy(np.ascontiguousarray(t.vals)).to(d)
    facs = [torch.from_numpy(np.ascontiguousarray(f)).to(d).to(dtype) for f in t.factors]
    return idx, vals, facs


def make_plan(t, **kw):
    idx, vals, facs = to_dev(t)
    p = Plan(idx, vals, t.dims, t.rank, **kw)
    return p, facs


def bf16_round(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.bfloat16).to(
        torch.float64).numpy()


def check_close(got, ref, refabs, tol, what=""):
    got = np.asarray(got, np.float64)
    diff = np.abs(got - ref)
    nref = np.linalg.norm(ref)
    nw = np.linalg.norm(got - ref) / nref if nref > 0 else np.linalg.norm(got - ref)
    assert nw <= tol, f"{what}: normwise error {nw:.3e} > {tol}"
    bad = diff > tol * refabs
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError(
            f"{what}: elementwise error {diff[tuple(i)]:.3e} > {tol} * "
            f"{refabs[tuple(i)]:.3e} at {tuple(i)} (got {got[tuple(i)]}, "
            f"ref {ref[tuple(i)]})")
    return nw, float((diff / np.where(refabs > 0, refabs, 1)).max())


def oracle_layout_records(t, order):
    """(nnz, N+1) int32 records of the oracle's layout: coords, value bits."""
    N = t.idx.shape[0]
    rec = np.empty((order.shape[0], N + 1), np.int32)
    rec[:, :N] = t.idx[:, order].T
    rec[:, N] = t.vals[order].view(np.int32)
    return rec


__all__ = ["FP32_TOL", "BF16_TOL", "say", "dev", "to_dev", "make_plan",
           "bf16_round", "check_close", "oracle_layout_records", "oracle", "_abi"]
