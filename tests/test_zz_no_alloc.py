"""The allocation-free CP-ALS sweep (cp_als_sweep_static: its scratch is a
static device array inside the library) against cp_als_sweep with a caller
buffer, through the C ABI: two calls in a row, the second on a smaller
tensor, each compared element by element (both run the same kernels in the
same order, so the results must be identical)."""
import numpy as np
import pytest
import torch

from gpu_common import _abi, dev, say, to_dev
from paper_2309_09131_amd import synthetic as syn
from paper_2309_09131_amd.api import Plan, _fdt, _ptr, _stream

pytestmark = pytest.mark.gpu


def _sweep_pair(dims, nnz, R, seed, dtype):
    say(f"static-scratch sweep: dims={dims} nnz={nnz} R={R} dtype={dtype}")
    t = syn.random_tensor(dims, nnz, R, seed, zipf_s=1.1)
    idx, vals, facs = to_dev(t, dtype)
    p = Plan(idx, vals, dims, R, g=256)
    d = dev()
    # reference: caller-provided scratch
    fa = [f.clone() for f in facs]
    mbuf = torch.empty((max(dims), R), dtype=torch.float32, device=d)
    lam_a = torch.empty(R, dtype=torch.float64, device=d)
    fit_a = torch.empty((), dtype=torch.float64, device=d)
    _abi.cp_als_sweep(p.handle, [_ptr(f) for f in fa], _fdt(fa), _ptr(mbuf), _ptr(lam_a),
                      _ptr(fit_a), _stream())
    # the allocation-free entry point
    fb = [f.clone() for f in facs]
    lam_b = torch.full((R,), -1.0, dtype=torch.float64, device=d)
    fit_b = torch.full((), -1.0, dtype=torch.float64, device=d)
    _abi.cp_als_sweep_static(p.handle, [_ptr(f) for f in fb], _fdt(fb), _ptr(lam_b),
                             _ptr(fit_b), _stream())
    torch.cuda.synchronize()
    for n in range(len(dims)):
        assert torch.equal(fa[n], fb[n]), f"factor {n} differs"
        assert not torch.equal(fb[n], facs[n]), f"factor {n} was not updated"
    assert torch.equal(lam_a, lam_b)
    assert torch.equal(fit_a, fit_b)
    assert np.isfinite(fit_b.item())
    return p


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_static_scratch_sweep_equals_caller_buffer_sweep(dtype):
    # first call: the larger tensor; second call: a smaller one, on the same
    # array, which still holds the first call's contents
    _sweep_pair((900, 700, 500), 60000, 32, 81, dtype)
    _sweep_pair((50, 40, 30, 20), 3000, 8, 82, dtype)


def test_static_scratch_size_limit_is_einval():
    # max_n I_n * R = 2^20 * 32 = 2^25 > 2^24 floats
    d = dev()
    dims = (1 << 20, 4, 4)
    idx = torch.stack([torch.arange(8, dtype=torch.int32, device=d) * 1000,
                       torch.arange(8, dtype=torch.int32, device=d) % 4,
                       torch.arange(8, dtype=torch.int32, device=d) % 3])
    vals = torch.ones(8, dtype=torch.float32, device=d)
    p = Plan(idx, vals, dims, 32, g=256)
    facs = [torch.ones((n, 32), dtype=torch.float32, device=d) for n in dims]
    lam = torch.empty(32, dtype=torch.float64, device=d)
    with pytest.raises(_abi.MttkrpError) as ei:
        _abi.cp_als_sweep_static(p.handle, [_ptr(f) for f in facs], _abi.F32, _ptr(lam), 0,
                                 _stream())
    assert ei.value.status == _abi.EINVAL
    assert "static scratch" in str(ei.value)
