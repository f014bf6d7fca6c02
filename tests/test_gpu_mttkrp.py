"""GPU parity of the plan, remap and per-mode MTTKRP against the FP64 oracle.

Integer work (layouts, remap targets, row pointers, shard tables, schedule)
must match bit for bit; floating point within 1e-5 (FP32) / 2e-2 (BF16),
normwise and elementwise relative to the |.|-sum M^abs.
"""
import numpy as np
import pytest
import torch

from gpu_common import (BF16_TOL, FP32_TOL, _abi, bf16_round, check_close,
                        dev, make_plan, oracle, oracle_layout_records, say,
                        to_dev)
from paper_2309_09131_amd import synthetic as syn
from paper_2309_09131_amd.api import Plan

pytestmark = pytest.mark.gpu

PLAN_CASES = [
    # dims, nnz, R, seed, distinct, zipf, g
    ((60, 50, 40), 3000, 16, 1, True, 0.0, 64),
    ((7, 5, 6), 150, 4, 2, False, 0.0, 16),          # duplicates
    ((40, 3, 30, 5), 2500, 8, 3, True, 1.2, 100),
    ((9, 2, 11, 3, 4), 900, 5, 4, False, 0.0, 32),
    ((300, 200), 5000, 3, 5, True, 1.1, 128),
    ((1, 40, 30), 600, 2, 6, True, 0.0, 50),          # I_0 = 1
]


@pytest.mark.parametrize("case", PLAN_CASES)
def test_plan_tables_bit_exact(case):
    dims, nnz, R, seed, distinct, zipf, g = case
    say("plan case", case)
    t = syn.random_tensor(dims, nnz, R, seed, distinct=distinct, zipf_s=zipf)
    p, _ = make_plan(t, g=g, workers=4)
    l0 = oracle.canonical_order(t.idx)
    layouts, perm, rps = oracle.remap_replay(dims, t.idx, l0)
    got = p.query(_abi.Q_LAYOUT)
    assert np.array_equal(got, oracle_layout_records(t, layouts[0]))
    N = len(dims)
    for n in range(N):
        assert np.array_equal(p.query(_abi.Q_PERM, n), perm[n]), n
        assert np.array_equal(p.query(_abi.Q_ROW_PTR, n), rps[n]), n
        m = p.info(_abi.INFO_M, n)
        sh = oracle.shards(dims[n], rps[n], m, g)
        tab = p.query(_abi.Q_SHARDS, n)
        assert np.array_equal(tab[:, 0], sh["start"])
        assert np.array_equal(tab[:, 1], sh["len"])
        assert np.array_equal(tab[:, 2], sh["ss"])
        bins, _ = oracle.lpt(sh["ss_shards"], 4)
        assert np.array_equal(p.query(_abi.Q_LPT, n), bins)
    # standalone remap walks the oracle's layouts and returns to L_0
    for n in range(1, N + 1):
        p.remap(n % N)
        assert np.array_equal(p.query(_abi.Q_LAYOUT),
                              oracle_layout_records(t, layouts[n])), n


# Morton codes wider than 31 bits: sorted in two slices
LOCALITY_CASES = PLAN_CASES + [((300000, 200000, 5000), 5000, 4, 31, True, 0.0, 64),
                               ((70000, 90000, 5000, 300), 6000, 4, 32, True, 1.1, 128)]


@pytest.mark.parametrize("case", LOCALITY_CASES)
def test_locality_order_plan_bit_exact(case):
    """The locality-order option: every layout, remap target and row pointer
    equal the oracle's (Morton order inside output rows), byte for byte,
    through a whole sweep of standalone remaps."""
    dims, nnz, R, seed, distinct, zipf, g = case
    say("locality plan case", case)
    t = syn.random_tensor(dims, nnz, R, seed, distinct=distinct, zipf_s=zipf)
    p, _ = make_plan(t, g=g, workers=4, flags=_abi.LOCALITY_ORDER)
    layouts, perm = oracle.locality_layouts(dims, t.idx)
    _, _, rps = oracle.remap_replay(dims, t.idx)
    N = len(dims)
    for n in range(N):
        assert np.array_equal(p.query(_abi.Q_PERM, n), perm[n]), n
        assert np.array_equal(p.query(_abi.Q_ROW_PTR, n), rps[n]), n
    for n in range(N + 1):
        if n:
            p.remap(n % N)
        assert np.array_equal(p.query(_abi.Q_LAYOUT),
                              oracle_layout_records(t, layouts[n])), n


MTT_CASES = [
    # dims, nnz, R, seed, distinct, zipf, g, factor dtype
    ((60, 50, 40), 3000, 16, 11, True, 0.0, 64),
    ((60, 50, 40), 3000, 32, 12, True, 1.2, 64),
    ((30, 20, 10), 1500, 64, 13, False, 0.0, 100),
    ((50, 40, 30), 2000, 17, 14, True, 0.0, 64),      # strided lanes
    ((20, 30, 25), 800, 1, 15, True, 0.0, 32),
    ((20, 30, 25), 800, 256, 16, True, 0.0, 128),
    ((40, 3, 30, 5), 2500, 8, 17, True, 1.2, 100),
    ((9, 2, 11, 3, 4), 900, 20, 18, False, 0.0, 32),
    ((300, 200), 5000, 12, 19, True, 1.1, 128),
    ((3, 2, 2, 3, 2, 2, 3, 2), 700, 16, 20, False, 0.0, 50),   # N = 8
    ((2000, 30, 20), 500, 16, 21, True, 0.0, 64),     # many empty rows
    ((50, 40, 30), 37, 16, 22, True, 0.0, 1024),      # nnz < 64
    ((4, 500, 300), 20000, 16, 23, True, 1.5, 64),    # rows over many shards
    ((3, 200, 100), 150000, 8, 24, False, 0.0, 2),    # ~75K partials: 3 levels
    ((60, 50, 2, 10, 9), 20000, 16, 25, True, 0.0, 64),  # a 2-index mode
    # packed records: L_2 stores 19 + 18 bits in two words, mode 1 straddling them
    ((300000, 200000, 5000), 5000, 16, 26, True, 0.0, 64),
    ((70000, 90000, 5000, 300), 6000, 32, 27, True, 1.1, 128),   # 17 + 17 + 13 + 9 bits
    # output rows from the row-start table: runs of 1024 positions crossing
    # 16 table blocks (strided lanes), and mostly single-nonzero rows, so that
    # nearly every step of a slot starts several rows
    ((100000, 50, 40), 20000, 20, 29, True, 0.0, 1024),
    ((200000, 64, 50), 30000, 32, 30, True, 0.0, 512),
]


def _oracle_all(t, facs64):
    return [oracle.mttkrp(t.dims, t.idx, t.vals, facs64, n, with_abs=True)
            for n in range(len(t.dims))]


@pytest.mark.parametrize("flags", [0, _abi.FUSED_REMAP, _abi.UNPACKED_RECORDS,
                                   _abi.LOCALITY_ORDER])
@pytest.mark.parametrize("case", MTT_CASES)
def test_mttkrp_all_modes_fp32(case, flags):
    dims, nnz, R, seed, distinct, zipf, g = case
    say("mttkrp fp32 case", case, "flags", flags)
    t = syn.random_tensor(dims, nnz, R, seed, distinct=distinct, zipf_s=zipf)
    p, facs = make_plan(t, g=g, flags=flags)
    outs = p.mttkrp_all_modes(facs)
    torch.cuda.synchronize()
    assert p.cur_mode == 0
    ref = _oracle_all(t, t.factors)
    for n in range(len(dims)):
        check_close(outs[n].cpu().numpy(), ref[n][0], ref[n][1], FP32_TOL, f"mode {n}")
    # deterministic: a second sweep is bit-identical
    outs2 = p.mttkrp_all_modes(facs)
    for a, b in zip(outs, outs2):
        assert torch.equal(a, b)
    # the layout is back in L_0 and byte-identical to the oracle's
    l0 = (oracle.locality_layouts(dims, t.idx)[0][0] if flags & _abi.LOCALITY_ORDER
          else oracle.canonical_order(t.idx))
    assert np.array_equal(p.query(_abi.Q_LAYOUT), oracle_layout_records(t, l0))


@pytest.mark.parametrize("case", [c for c in MTT_CASES if c[2] % 8 == 0 or c[2] in (1, 17, 20, 12)])
def test_mttkrp_bf16_factors(case):
    dims, nnz, R, seed, distinct, zipf, g = case
    say("mttkrp bf16 case", case)
    t = syn.random_tensor(dims, nnz, R, seed, distinct=distinct, zipf_s=zipf)
    idx, vals, facs = to_dev(t, torch.bfloat16)
    p = Plan(idx, vals, dims, R, g=g, flags=_abi.FUSED_REMAP if seed % 2 else 0)
    outs = p.mttkrp_all_modes(facs)
    ref32 = _oracle_all(t, t.factors)                        # includes storage error
    refb = _oracle_all(t, [bf16_round(f) for f in t.factors])  # accumulation only
    for n in range(len(dims)):
        got = outs[n].cpu().numpy()
        check_close(got, ref32[n][0], ref32[n][1], BF16_TOL, f"bf16 vs fp32 mode {n}")
        check_close(got, refb[n][0], refb[n][1], FP32_TOL, f"bf16 vs bf16-oracle {n}")


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_integer_inputs_bit_exact(dtype):
    """Integer values in [1,4], factors in [-2,2]: every partial sum is an
    integer below 2^24, so any summation order gives the exact result."""
    for dims, R, g in [((40, 30, 20), 16, 64), ((12, 9, 7, 5), 32, 50),
                       ((30, 25), 24, 40)]:
        t = syn.random_tensor(dims, 1500, R, 31, distinct=False, int_values=True)
        idx, vals, facs = to_dev(t, dtype)
        p = Plan(idx, vals, dims, R, g=g)
        outs = p.mttkrp_all_modes(facs)
        for n in range(len(dims)):
            ref = oracle.mttkrp(dims, t.idx, t.vals, t.factors, n)
            assert np.array_equal(outs[n].cpu().numpy().astype(np.float64), ref), (dims, n)


@pytest.mark.parametrize("extra", [0, _abi.FUSED_REMAP])
def test_single_mode_fused_and_unfused_and_state(extra):
    t = syn.random_tensor((80, 60, 40, 30), 5000, 16, 41, zipf_s=1.1)
    p, facs = make_plan(t, g=128, flags=_abi.NO_IMPLICIT_REMAP | extra)
    ref = _oracle_all(t, t.factors)
    out = p.mttkrp_mode(0, facs, fuse_remap=False)
    check_close(out.cpu().numpy(), ref[0][0], ref[0][1], FP32_TOL, "unfused mode 0")
    assert p.cur_mode == 0
    with pytest.raises(_abi.MttkrpError) as ei:
        p.mttkrp_mode(2, facs)
    assert ei.value.status == _abi.ESTATE
    for n in range(4):
        out = p.mttkrp_mode(n, facs, fuse_remap=True)
        check_close(out.cpu().numpy(), ref[n][0], ref[n][1], FP32_TOL, f"fused {n}")
    assert p.cur_mode == 0
    # implicit remap when allowed
    q, facs2 = make_plan(t, g=128)
    out = q.mttkrp_mode(3, facs2, fuse_remap=False)
    assert q.cur_mode == 3
    check_close(out.cpu().numpy(), ref[3][0], ref[3][1], FP32_TOL, "implicit")


def test_out_of_range_index_is_erange():
    d = dev()
    idx = torch.tensor([[0, 1, 5], [0, 1, 2]], dtype=torch.int32, device=d)
    vals = torch.ones(3, dtype=torch.float32, device=d)
    with pytest.raises(_abi.MttkrpError) as ei:
        Plan(idx, vals, (5, 3), 4)
    assert ei.value.status == _abi.ERANGE


def test_empty_tensor_gives_zero_outputs():
    d = dev()
    idx = torch.zeros((3, 0), dtype=torch.int32, device=d)
    vals = torch.zeros(0, dtype=torch.float32, device=d)
    p = Plan(idx, vals, (5, 4, 3), 8)
    facs = [torch.randn(n, 8, device=d) for n in (5, 4, 3)]
    outs = p.mttkrp_all_modes(facs)
    for o in outs:
        assert torch.count_nonzero(o) == 0


@pytest.mark.parametrize("flags", [0, _abi.FUSED_REMAP])
def test_one_output_buffer_for_every_mode(flags):
    """Callers may pass the same buffer as the output of every mode: the
    split-row reduction of one pass (on the side stream) must finish before
    the next pass writes the buffer.  After the sweep the buffer holds the
    last mode's result, equal to the oracle's."""
    dims, R = (400, 300, 200), 32
    t = syn.random_tensor(dims, 60000, R, 33, zipf_s=1.4)
    p, facs = make_plan(t, g=32, flags=flags)   # many rows split across shards
    assert all(p.info(_abi.INFO_NSPLIT, n) > 0 for n in range(3))
    big = torch.empty(max(dims) * R, dtype=torch.float32, device=facs[0].device)
    outs = [big[:d * R].view(d, R) for d in dims]
    for _ in range(3):
        big.fill_(float("nan"))
        p.mttkrp_all_modes(facs, outs)
        torch.cuda.synchronize()
        ref, rabs = oracle.mttkrp(dims, t.idx, t.vals, t.factors, 2, with_abs=True)
        check_close(outs[2].cpu().numpy(), ref, rabs, FP32_TOL, "last mode")


def _random_case(seed):
    """A small tensor of random shape: 2 to 8 modes, some tiny and some with
    more rows than nonzeros (empty rows), any shard size (1 up to 1024, not
    only multiples of 64), ranks for every lane form, and a record form."""
    rng = np.random.default_rng(1000 + seed)
    N = int(rng.choice([2, 3, 3, 4, 4, 5, 6, 8]))
    dims = tuple(int(rng.choice([1, 2, 5, 37, 300, 2000, 70000])) for _ in range(N))
    if max(dims) == 1:
        dims = dims[:-1] + (40,)
    nnz = int(rng.integers(1, 4000))
    distinct = bool(rng.random() < 0.5)
    if distinct:
        nnz = min(nnz, int(np.prod(dims, dtype=np.float64) // 2) + 1)
    R = int(rng.choice([1, 3, 4, 8, 12, 16, 20, 32, 48, 64]))
    g = int(rng.choice([1, 3, 7, 63, 64, 65, 100, 257, 1024]))
    zipf = float(rng.choice([0.0, 1.3]))
    flags = int(rng.choice([0, _abi.FUSED_REMAP, _abi.UNPACKED_RECORDS]))
    return dims, nnz, R, distinct, zipf, g, flags


@pytest.mark.parametrize("seed", range(16))
def test_random_shapes_rows_and_layouts(seed):
    """Randomly shaped small tensors: every mode's MTTKRP against the oracle
    and every layout of a full remap cycle byte-exact, so that the output
    rows the kernels recover from the row-start tables (shards that start
    and end anywhere in a 64-position block, one-nonzero shards, empty rows)
    and the records the remap rewrites are both checked."""
    dims, nnz, R, distinct, zipf, g, flags = _random_case(seed)
    say("random case", seed, dims, nnz, R, distinct, zipf, g, flags)
    t = syn.random_tensor(dims, nnz, R, 500 + seed, distinct=distinct, zipf_s=zipf)
    p, facs = make_plan(t, g=g, flags=flags)
    outs = p.mttkrp_all_modes(facs)
    torch.cuda.synchronize()
    N = len(dims)
    for n in range(N):
        ref, rabs = oracle.mttkrp(dims, t.idx, t.vals, t.factors, n, with_abs=True)
        check_close(outs[n].cpu().numpy(), ref, rabs, FP32_TOL, f"mode {n}")
    layouts, _, _ = oracle.remap_replay(dims, t.idx)
    assert p.cur_mode == 0
    assert np.array_equal(p.query(_abi.Q_LAYOUT), oracle_layout_records(t, layouts[0]))
    for n in range(1, N + 1):
        p.remap(n % N)
        assert np.array_equal(p.query(_abi.Q_LAYOUT),
                              oracle_layout_records(t, layouts[n])), n


@pytest.mark.parametrize("dims, words", [((50000, 40000, 30000), 1),
                                         ((300000, 200000, 5000), 2),
                                         ((70000, 90000, 5000, 300), 2),
                                         ((3, 2, 2, 3, 2, 2, 3, 2), 5)])
def test_record_bytes_and_layout(dims, words):
    """Stored records are (packed words + 1) * 4 bytes, N * 4 unpacked (a
    layout's records omit its own output coordinate); both forms give the
    oracle's layout for every mode."""
    say("record width", dims)
    t = syn.random_tensor(dims, 3000, 8, 28, distinct=False)
    l0 = oracle.canonical_order(t.idx)
    layouts, _, _ = oracle.remap_replay(dims, t.idx, l0)
    N = len(dims)
    for flags, nbytes in ((0, 4 * (words + 1)), (_abi.UNPACKED_RECORDS, 4 * N)):
        p, _ = make_plan(t, g=64, flags=flags)
        assert p.info(_abi.INFO_RECORD_BYTES) == nbytes
        for n in range(N + 1):
            assert np.array_equal(p.query(_abi.Q_LAYOUT),
                                  oracle_layout_records(t, layouts[n])), (flags, n)
            p.remap((n + 1) % N)


# N = 3 Zipf, N = 4, N = 5, N = 2, rows over many shards, three reduction levels
RESIDENT_CASES = [MTT_CASES[1], MTT_CASES[6], MTT_CASES[7], MTT_CASES[8], MTT_CASES[12],
                  MTT_CASES[13]]


def _resident_masks(N):
    R = _abi.RESIDENT_LAYOUT
    masks = [R(0), R(N - 1), sum(R(n) for n in range(N))]
    if N > 2:
        masks.append(R(1) | R(N - 1))
    return masks


@pytest.mark.parametrize("extra", [0, _abi.FUSED_REMAP])
@pytest.mark.parametrize("case", RESIDENT_CASES)
def test_resident_layouts_give_the_same_results(case, extra):
    """Plans that keep some or all layouts resident: the default plan's
    outputs bit for bit over repeated sweeps, the oracle's layouts at every
    step of a standalone remap walk, and implicit remaps to single modes."""
    dims, nnz, R, seed, distinct, zipf, g = case
    say("resident case", case, "extra", extra)
    t = syn.random_tensor(dims, nnz, R, seed, distinct=distinct, zipf_s=zipf)
    N = len(dims)
    base, facs = make_plan(t, g=g, flags=extra)
    ref = [o.clone() for o in base.mttkrp_all_modes(facs)]
    layouts, _, _ = oracle.remap_replay(dims, t.idx)
    for mask in _resident_masks(N):
        p, _ = make_plan(t, g=g, flags=extra | mask)
        assert np.array_equal(p.query(_abi.Q_LAYOUT), oracle_layout_records(t, layouts[0]))
        for _ in range(2):
            outs = p.mttkrp_all_modes(facs)
            torch.cuda.synchronize()
            assert p.cur_mode == 0
            for n in range(N):
                assert torch.equal(outs[n], ref[n]), (mask, n)
        for n in range(1, N + 1):
            p.remap(n % N)
            assert np.array_equal(p.query(_abi.Q_LAYOUT),
                                  oracle_layout_records(t, layouts[n])), (mask, n)
        # implicit remaps: the last mode, then the first again
        o = p.mttkrp_mode(N - 1, facs, fuse_remap=False)
        assert torch.equal(o, ref[N - 1])
        o = p.mttkrp_mode(0, facs)
        assert torch.equal(o, ref[0]) and p.cur_mode == 1 % N


def test_resident_layouts_cp_als_and_loss_unchanged():
    """CP-ALS sweeps and the loss with its gradients on a plan with resident
    layouts equal those of the default plan bit for bit."""
    t = syn.random_tensor((40, 3, 30, 5), 2500, 8, 33, zipf_s=1.2)
    R = _abi.RESIDENT_LAYOUT
    base, facs = make_plan(t, g=100)
    res, _ = make_plan(t, g=100, flags=R(0) | R(2))
    fa = [f.clone() for f in facs]
    fb = [f.clone() for f in facs]
    for _ in range(2):
        la, ta = base.cp_als_sweep(fa)
        lb, tb = res.cp_als_sweep(fb)
    torch.cuda.synchronize()
    assert torch.equal(la, lb) and torch.equal(ta, tb)
    for a, b in zip(fa, fb):
        assert torch.equal(a, b)
    u = [torch.rand_like(f) for f in facs]
    l1, g1 = base.cp_loss_grad(u)
    l2, g2 = res.cp_loss_grad(u)
    torch.cuda.synchronize()
    assert l1.item() == l2.item()
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
