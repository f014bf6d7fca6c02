"""Host-side checks of the C ABI (no GPU needed): every symbol the header
declares is exported, and argument errors are reported as status codes
before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2309_09131_amd import _abi, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        build.build_lib(force=False)
    return _abi.load()


def header_functions():
    src = open(os.path.join(ROOT, "include", "mttkrp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(",
                                 src, flags=re.M)))


def test_header_symbols_exported(lib):
    names = header_functions()
    assert len(names) >= 14, names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(_abi.SYMBOLS)


def test_workspace_argument_errors(lib):
    ok = _abi.mttkrp_plan_workspace(3, (10, 20, 30), 1000, 16)
    assert ok > 1000 * 16 * 2
    for args in [(1, (10,), 5, 4), (9, (2,) * 9, 5, 4), (3, (10, 20, 30), 5, 0),
                 (3, (10, 20, 30), 5, 257), (3, (10, 0, 30), 5, 4),
                 (3, (10, 20, 30), -1, 4), (3, (10, 20, 30), 1 << 31, 4)]:
        with pytest.raises(_abi.MttkrpError) as ei:
            _abi.mttkrp_plan_workspace(*args)
        assert ei.value.status == _abi.EINVAL, args
    with pytest.raises(_abi.MttkrpError):
        _abi.mttkrp_plan_workspace(3, (10, 20, 30), 5, 4, _abi.make_opts(g=-1))


def test_nnz_limit_keeps_kernel_indices_in_int32(lib):
    """Kernels index nonzeros with 32-bit integers and may step a few hundred
    past a shard's end before clamping, so the plan refuses nnz above
    MTTKRP_MAX_NNZ = 2^31 - 2^20 (sizes only: no device work)."""
    assert _abi.MAX_NNZ == (1 << 31) - (1 << 20)
    dims = (1 << 20, 1 << 20, 1 << 20)
    for nnz in ((1 << 31) - 1, (1 << 31) - 256, _abi.MAX_NNZ + 1):
        with pytest.raises(_abi.MttkrpError) as ei:
            _abi.mttkrp_plan_workspace(3, dims, nnz, 16)
        assert ei.value.status == _abi.EINVAL, nnz
        assert str(_abi.MAX_NNZ) in str(ei.value)
    need = _abi.mttkrp_plan_workspace(3, dims, _abi.MAX_NNZ, 16)
    assert need > 2 * _abi.MAX_NNZ * 12


def test_plan_argument_errors_before_device_work(lib):
    dims = (10, 20, 30)
    need = _abi.mttkrp_plan_workspace(3, dims, 100, 8)
    # NULL workspace, misaligned workspace, NULL inputs, small workspace
    with pytest.raises(_abi.MttkrpError) as ei:
        _abi.mttkrp_plan(3, dims, 100, 4096, 8192, 8, None, 0, need)
    assert ei.value.status == _abi.EINVAL
    with pytest.raises(_abi.MttkrpError) as ei:
        _abi.mttkrp_plan(3, dims, 100, 4096, 8192, 8, None, 4096 + 8, need)
    assert ei.value.status == _abi.EINVAL
    with pytest.raises(_abi.MttkrpError) as ei:
        _abi.mttkrp_plan(3, dims, 100, 0, 8192, 8, None, 4096, need)
    assert ei.value.status == _abi.EINVAL
    with pytest.raises(_abi.MttkrpError) as ei:
        _abi.mttkrp_plan(3, dims, 100, 4096, 8192, 8, None, 4096, need - 1)
    assert ei.value.status == _abi.ENOMEM
    assert "needs" in _abi.mttkrp_last_error(None)


def test_calls_on_null_plan_are_einval(lib):
    for fn, args in [(lib.mttkrp_mode, (None, 0, None, 0, None, 1, None)),
                     (lib.mttkrp_all_modes, (None, None, 0, None, None)),
                     (lib.remap, (None, 0, None)),
                     (lib.cp_loss_grad, (None, None, 0, None, None, None, None)),
                     (lib.cp_als_sweep, (None, None, 0, None, None, None, None)),
                     (lib.cp_als, (None, None, 0, None, None, 1, 0.0, None, None, None, None)),
                     (lib.mttkrp_plan_destroy, (None,))]:
        assert fn(*args) == _abi.EINVAL
    assert lib.mttkrp_status_str(_abi.ESTATE).decode().startswith("tensor")


def test_status_strings(lib):
    for st in range(6):
        assert len(_abi.mttkrp_status_str(st)) > 0


def _align(x):
    return (x + 255) & ~255


# A record of layout L_m holds the coordinates other than c_m; the packed
# width is the widest layout's, at least 2 words from four modes and N - 3
# from five.
@pytest.mark.parametrize("dims, packed_words", [
    ((50000, 40000, 30000), 1),                 # 16 + 16 + 15 bits: at most 32 stored
    ((300000, 200000, 5000), 2),                # 19 + 18 + 13: 37 bits stored in L_2
    ((1 << 30, 1 << 30, 1 << 30), 2),           # 60 bits stored: no saving
    ((70000, 90000, 5000, 300), 2),             # 47 bits stored in L_3
    ((1000000, 500000, 20000, 2000), 2),        # 20 + 19 + 15 + 11: 54 bits in L_3
    ((2000000, 1000000, 100000, 5000, 500), 3),  # 71 bits stored in L_4
    ((1, 5, 1), 1),                             # 0-bit modes
])
def test_record_width_from_dimensions(lib, dims, packed_words):
    """The stored record is (packed coordinate words + 1) * 4 bytes; with
    MTTKRP_UNPACKED_RECORDS it is N * 4 (one word per stored coordinate and
    the value).  The two record buffers of the workspace, and the remap's
    per-region row ids (regions sized from the width), depend on it."""
    nnz, N = 100003, len(dims)
    packed = _abi.mttkrp_plan_workspace(N, dims, nnz, 16)
    wide = _abi.mttkrp_plan_workspace(N, dims, nnz, 16,
                                      _abi.make_opts(flags=_abi.UNPACKED_RECORDS))
    assert wide - packed == _width_delta(dims, nnz, N - 1, packed_words)


def _remap_rt(W, small):
    """Records per thread of the standalone remap (the library's rule)."""
    per = 256 * (4 * (W + 1) + 4)
    if small:
        return min(16, 72 * 1024 // per)
    return min(32 if W + 1 == 2 else 24 if W + 1 == 3 else 16, 96 * 1024 // per)


def _width_delta(dims, nnz, w_wide, w_packed):
    """Workspace bytes that depend on the record width: the two record
    buffers, and each layout's per-region row ids of its remap (one region
    of 64 * RT records per remap wave, RT from the width)."""
    N = len(dims)
    rec = lambda w: _align(nnz * 4 * (w + 1))
    d = 2 * (rec(w_wide) - rec(w_packed))
    for n in range(N):
        small = dims[(n + 1) % N] <= 1 << 16
        for w, sgn in ((w_wide, 1), (w_packed, -1)):
            rb = 256 * _remap_rt(w, small)
            d += sgn * _align(max(4 * -(-nnz // rb), 1) * 64 * 4)
    return d


def _stored_words(dims):
    """Packed words from the width rule, written out independently."""
    N = len(dims)
    bits = [max(int(d - 1).bit_length(), 0) for d in dims]
    w = max((sum(bits) - bits[m] + 31) // 32 for m in range(N))
    wmin = N - 3 if N >= 5 else (2 if N == 4 else 1)
    return max(w, wmin, 1)


def test_record_width_rule_over_many_shapes(lib):
    """The packed width for random shapes of 2 to 8 modes follows the rule:
    the widest layout's stored coordinates, rounded up to the narrowest
    compiled width."""
    rng = np.random.default_rng(3)
    nnz = 4099
    for _ in range(60):
        N = int(rng.integers(2, 9))
        dims = tuple(int(x) for x in rng.integers(1, 1 << int(rng.integers(1, 31)), N))
        packed = _abi.mttkrp_plan_workspace(N, dims, nnz, 8)
        wide = _abi.mttkrp_plan_workspace(N, dims, nnz, 8,
                                          _abi.make_opts(flags=_abi.UNPACKED_RECORDS))
        assert wide - packed == _width_delta(dims, nnz, N - 1, _stored_words(dims)), dims


def test_python_constants_match_header():
    """Flags, query ids, info keys and profiling ids in the binding carry the
    header's values."""
    src = open(os.path.join(ROOT, "include", "mttkrp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    vals = {m.group(1): int(m.group(2))
            for m in re.finditer(r"#define\s+MTTKRP_([A-Z_0-9]+)\s+(\d+)u?\b", src)}
    vals.update({m.group(1): int(m.group(2))
                 for m in re.finditer(r"\bMTTKRP_([A-Z_0-9]+)\s*=\s*(\d+)", src)})
    pairs = {"NO_IMPLICIT_REMAP": _abi.NO_IMPLICIT_REMAP, "NATURAL_ORDER": _abi.NATURAL_ORDER,
             "FUSED_REMAP": _abi.FUSED_REMAP, "UNPACKED_RECORDS": _abi.UNPACKED_RECORDS,
             "GATHER_ONLY": _abi.GATHER_ONLY, "LOCALITY_ORDER": _abi.LOCALITY_ORDER,
             "Q_LAYOUT": _abi.Q_LAYOUT, "Q_PERM": _abi.Q_PERM, "Q_ROW_PTR": _abi.Q_ROW_PTR,
             "Q_SHARDS": _abi.Q_SHARDS, "Q_LPT": _abi.Q_LPT,
             "INFO_CUR_MODE": _abi.INFO_CUR_MODE, "INFO_NSHARDS": _abi.INFO_NSHARDS,
             "INFO_NSUPER": _abi.INFO_NSUPER, "INFO_NSPLIT": _abi.INFO_NSPLIT,
             "INFO_G": _abi.INFO_G, "INFO_M": _abi.INFO_M, "INFO_RIDGE": _abi.INFO_RIDGE,
             "INFO_RECORD_BYTES": _abi.INFO_RECORD_BYTES,
             "PROF_MTTKRP": _abi.PROF_MTTKRP, "PROF_REMAP": _abi.PROF_REMAP,
             "PROF_RESID": _abi.PROF_RESID, "PROF_LOSS": _abi.PROF_LOSS,
             "MAX_NNZ": _abi.MAX_NNZ, "MAX_MODES": _abi.MAX_MODES,
             "STATIC_MBUF_FLOATS": _abi.STATIC_MBUF_FLOATS,
             "F32": _abi.F32, "BF16": _abi.BF16, "OK": _abi.OK, "EINVAL": _abi.EINVAL,
             "ERANGE": _abi.ERANGE, "ENOMEM": _abi.ENOMEM, "ESTATE": _abi.ESTATE,
             "EHIP": _abi.EHIP}
    for name, v in pairs.items():
        assert vals.get(name) == v, (name, vals.get(name), v)


def test_resident_layouts_workspace_and_argument_check(lib):
    """Each resident layout adds one buffer of stored records to the
    workspace (8-byte records here: at most 10 stored coordinate bits in one
    word); a resident bit at or above nmodes is EINVAL."""
    dims, nnz = (10, 20, 30), 100000
    base = _abi.mttkrp_plan_workspace(3, dims, nnz, 16)
    for mask, k in ((_abi.RESIDENT_LAYOUT(0), 1), (_abi.RESIDENT_LAYOUT(2), 1),
                    (_abi.RESIDENT_LAYOUT(0) | _abi.RESIDENT_LAYOUT(1) | _abi.RESIDENT_LAYOUT(2),
                     3)):
        ws = _abi.mttkrp_plan_workspace(3, dims, nnz, 16, _abi.make_opts(flags=mask))
        extra = ws - base
        assert k * nnz * 8 <= extra <= k * (nnz * 8 + 256), (mask, extra)
    with pytest.raises(_abi.MttkrpError) as ei:
        _abi.mttkrp_plan_workspace(3, dims, nnz, 16, _abi.make_opts(flags=_abi.RESIDENT_LAYOUT(3)))
    assert ei.value.status == _abi.EINVAL
