"""GPU parity of the sampled CP loss (forward, adjoint, autograd) and of the
CP-ALS sweep against the FP64 oracle."""
import numpy as np
import pytest
import torch

from gpu_common import (BF16_TOL, FP32_TOL, _abi, bf16_round, check_close,
                        dev, make_plan, oracle, say, to_dev)
from paper_2309_09131_amd import synthetic as syn
from paper_2309_09131_amd.api import Plan, cp_loss

pytestmark = pytest.mark.gpu

LOSS_CASES = [((60, 50, 40), 4000, 16, 51, 64), ((40, 3, 30, 5), 2500, 32, 52, 100),
              ((200, 150, 100), 20000, 64, 53, 256), ((30, 25, 20), 1000, 17, 54, 64),
              ((9, 2, 11, 3, 4), 900, 8, 55, 32), ((300, 200), 6000, 32, 56, 128),
              ((3, 2, 2, 3, 2, 2, 3, 2), 600, 8, 57, 50)]


def _loss_case(case, flags=0):
    dims, nnz, R, seed, g = case
    t = syn.random_tensor(dims, nnz, R, seed, factors="uniform")
    idx, vals, facs = to_dev(t)
    return t, Plan(idx, vals, dims, R, g=g, flags=flags), facs


def _grad_ref(t, facs64):
    """Oracle gradient and an |.| scale: -2 * MTTKRP with values rho."""
    N = len(t.dims)
    m = np.zeros(t.nnz)
    mabs = np.zeros(t.nnz)
    for r in range(t.rank):
        p = np.ones(t.nnz)
        for n in range(N):
            p = p * facs64[n][t.idx[n], r]
        m += p
        mabs += np.abs(p)
    rho = t.vals.astype(np.float64) - m
    refs = []
    for k in range(N):
        g, _ = oracle.mttkrp(t.dims, t.idx, rho, facs64, k, with_abs=True)
        _, gabs = oracle.mttkrp(t.dims, t.idx, np.abs(t.vals) + mabs, facs64, k,
                                with_abs=True)
        refs.append((-2.0 * g, 2.0 * gabs))
    return refs


@pytest.mark.parametrize("flags", [0, _abi.FUSED_REMAP, _abi.LOCALITY_ORDER])
@pytest.mark.parametrize("case", LOSS_CASES)
def test_loss_and_gradient_match_oracle(case, flags):
    say("loss case", case, "flags", flags)
    t, p, facs = _loss_case(case, flags)
    f64 = [f.astype(np.float64) for f in t.factors]
    L_ref, G_ref = oracle.cp_loss_grad(t.dims, t.idx, t.vals, f64)
    p.remap(1 % len(t.dims))                 # start away from L_0
    loss, grads = p.cp_loss_grad(facs)
    torch.cuda.synchronize()
    assert p.cur_mode == 1 % len(t.dims)     # N passes end where they began
    assert abs(loss.item() - L_ref) <= FP32_TOL * abs(L_ref)
    refs = _grad_ref(t, f64)
    for k in range(len(t.dims)):
        g = grads[k].cpu().numpy()
        # second route: the oracle's own gradient routine
        assert np.linalg.norm(g - G_ref[k]) <= FP32_TOL * np.linalg.norm(G_ref[k])
        check_close(g, refs[k][0], refs[k][1], FP32_TOL, f"grad {k}")
    # bit-identical when repeated
    loss2, grads2 = p.cp_loss_grad(facs)
    assert loss2.item() == loss.item()
    for a, b in zip(grads, grads2):
        assert torch.equal(a, b)


@pytest.mark.parametrize("flags", [0, _abi.FUSED_REMAP])
@pytest.mark.parametrize("case", LOSS_CASES)
def test_joint_loss_equals_loss_only_pass(case, flags):
    """Loss and gradients together take the loss from the first residual
    pass: the same value, bit for bit, as the loss pass alone, and the same
    gradients as the gradient-only passes."""
    t, p, facs = _loss_case(case, flags)
    p.remap(len(t.dims) - 1)                 # start away from L_0
    l_only, _ = p.cp_loss_grad(facs, grads=False)
    l_joint, g_joint = p.cp_loss_grad(facs)
    _, g_only = p.cp_loss_grad(facs, loss=False)
    torch.cuda.synchronize()
    assert p.cur_mode == len(t.dims) - 1
    assert l_joint.item() == l_only.item(), (l_joint.item(), l_only.item())
    for a, b in zip(g_joint, g_only):
        assert torch.equal(a, b)


def test_gpu_forward_central_difference_matches_gpu_gradient():
    """The loss is exactly quadratic in any single factor entry, so a large
    step (h = 0.25) swamps FP32 rounding without truncation error."""
    t, p, facs = _loss_case(((50, 40, 30), 3000, 16, 61, 64))
    _, grads = p.cp_loss_grad(facs, loss=False)
    rng = np.random.default_rng(3)
    h = 0.25
    for _ in range(12):
        k = int(rng.integers(0, 3))
        i = int(rng.choice(t.idx[k]))
        r = int(rng.integers(0, 16))
        fp = [f.clone() for f in facs]
        fm = [f.clone() for f in facs]
        fp[k][i, r] += h
        fm[k][i, r] -= h
        lp, _ = p.cp_loss_grad(fp, grads=False)
        lm, _ = p.cp_loss_grad(fm, grads=False)
        fd = (lp.item() - lm.item()) / (2 * h)
        g = grads[k][i, r].item()
        assert abs(fd - g) <= 1e-3 * max(1.0, abs(g)), (k, i, r, fd, g)


def test_autograd_function_scales_by_upstream_gradient():
    t, p, facs = _loss_case(((40, 30, 20), 2000, 16, 71, 64))
    fr = [f.clone().requires_grad_(True) for f in facs]
    loss = cp_loss(p, fr)
    assert loss.dtype == torch.float64 and loss.requires_grad
    (3.0 * loss).backward()
    L_ref, G_ref = oracle.cp_loss_grad(t.dims, t.idx, t.vals, t.factors)
    assert abs(loss.item() - L_ref) <= FP32_TOL * L_ref
    for k in range(3):
        g = fr[k].grad.cpu().numpy()
        assert np.linalg.norm(g - 3.0 * G_ref[k]) <= FP32_TOL * 3.0 * np.linalg.norm(G_ref[k])
    # only the factors that ask for gradients get them
    fr2 = [facs[0].clone().requires_grad_(True), facs[1], facs[2]]
    cp_loss(p, fr2).backward()
    assert fr2[0].grad is not None
    # no factor needs a gradient: the loss pass alone, the same value
    with torch.no_grad():
        l0 = cp_loss(p, facs)
    assert not l0.requires_grad and l0.item() == loss.item()
    # BF16 factors get BF16 gradients
    fb = [f.clone().to(torch.bfloat16).requires_grad_(True) for f in facs]
    cp_loss(p, fb).backward()
    assert all(f.grad is not None and f.grad.dtype == torch.bfloat16 for f in fb)


def test_loss_at_planted_truth_matches_noise_level():
    rng = np.random.default_rng(9)
    dims, R, nnz = (400, 300, 200), 8, 60000
    true = [rng.random((d, R)).astype(np.float32) for d in dims]
    t = syn.random_tensor(dims, nnz, R, 81)
    m = np.zeros(nnz)
    for r in range(R):
        m += true[0][t.idx[0], r].astype(np.float64) * true[1][t.idx[1], r] * true[2][t.idx[2], r]
    sigma = 0.01 * np.sqrt(np.mean(m * m))
    x = (m + sigma * rng.standard_normal(nnz)).astype(np.float32)
    d = dev()
    p = Plan(torch.from_numpy(t.idx).to(d), torch.from_numpy(x).to(d), dims, R, g=256)
    loss, _ = p.cp_loss_grad([torch.from_numpy(a).to(d) for a in true], grads=False)
    expect = nnz * sigma ** 2
    # FP32 model values carry ~1e-7 relative error, far below sigma = 1e-2 RMS
    assert abs(loss.item() - expect) < 5 * np.sqrt(2.0 / nnz) * expect + 1e-3 * expect


ALS_CASES = [((60, 50, 40), 5000, 8, 91, 64), ((30, 4, 25, 20), 4000, 16, 92, 100),
             ((80, 70, 60, 10, 5), 8000, 16, 93, 128), ((120, 100), 3000, 5, 94, 64),
             # R > 64: the update's staged form (W read from memory)
             ((120, 100, 90), 20000, 72, 96, 128)]


@pytest.mark.parametrize("case", ALS_CASES)
def test_cp_als_sweep_fp32(case):
    dims, nnz, R, seed, g = case
    say("als fp32 case", case)
    t = syn.random_tensor(dims, nnz, R, seed)
    idx, vals, facs = to_dev(t)
    p = Plan(idx, vals, dims, R, g=g)
    lam, fit = p.cp_als_sweep(facs)
    of, olam, ofit, ridge, _ = oracle.cp_als_sweep(dims, t.idx, t.vals, t.factors)
    assert ridge == 0 and p.info(_abi.INFO_RIDGE) == 0
    assert p.cur_mode == 0
    assert np.allclose(lam.cpu().numpy(), olam, rtol=1e-5, atol=0)
    for n in range(len(dims)):
        a = facs[n].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(a - of[n]) <= 1e-5 * np.linalg.norm(of[n]), n
        # elementwise, against the largest magnitude of the same column
        # (columns are normalised; an element's error comes from its row of
        # M_n times V^-1, whose size the column scale bounds)
        colmax = np.abs(of[n]).max(axis=0)
        err = np.abs(a - of[n]) / np.where(colmax > 0, colmax, 1.0)
        assert err.max() <= 1e-5, (n, err.max(), np.unravel_index(err.argmax(), err.shape))
    assert abs(fit.item() - ofit) <= 1e-6, (fit.item(), ofit)


@pytest.mark.parametrize("case", ALS_CASES[:3])
def test_cp_als_sweep_bf16(case):
    dims, nnz, R, seed, g = case
    say("als bf16 case", case)
    t = syn.random_tensor(dims, nnz, R, seed)
    idx, vals, facs = to_dev(t, torch.bfloat16)
    p = Plan(idx, vals, dims, R, g=g)
    lam, fit = p.cp_als_sweep(facs)
    of, olam, ofit, _, _ = oracle.cp_als_sweep(dims, t.idx, t.vals,
                                               [bf16_round(f) for f in t.factors])
    assert np.allclose(lam.cpu().numpy(), olam, rtol=BF16_TOL, atol=0)
    for n in range(len(dims)):
        a = facs[n].float().cpu().numpy().astype(np.float64)
        assert np.linalg.norm(a - of[n]) <= BF16_TOL * np.linalg.norm(of[n]), n
        colmax = np.abs(of[n]).max(axis=0)
        if n == 0:
            # the first update starts from the same factors on both sides:
            # the stored value is the BF16 rounding of an FP64 value within
            # FP32 accumulation error of the oracle's, so it is at most one
            # BF16 ulp (2^-8 relative; half an ulp for exact nearest) away
            assert np.all(np.abs(a - of[n]) <= 2.0 ** -8 * np.abs(of[n]) + 1e-5 * colmax), n
        else:
            # later modes see the BF16-stored earlier updates, the oracle the
            # FP64 ones: BF16-level differences, elementwise per column
            assert np.all(np.abs(a - of[n]) <= BF16_TOL * colmax), n
    assert abs(fit.item() - ofit) <= BF16_TOL


def _sum_of_squares(n):
    """n as a sum of at most four integer squares (Lagrange): a list of the
    roots, largest first."""
    import math

    def three(m):
        a = math.isqrt(m)
        while a >= 0:
            r = m - a * a
            b = math.isqrt(r)
            while b >= 0 and 2 * b * b >= r:
                c = math.isqrt(r - b * b)
                if c * c == r - b * b:
                    return [a, b, c]
                b -= 1
            a -= 1
        return None

    a = math.isqrt(n)
    while a >= 0:
        t = three(n - a * a)
        if t is not None:
            return [x for x in [a] + t if x > 0]
        a -= 1
    raise AssertionError(n)


def _bf16_tie_tensor(I0=64, I1=24, I2=24, R=16, seed=7):
    """A 3-mode tensor whose first CP-ALS mode update has exactly known FP64
    values, several of them exactly halfway between two BF16 numbers.

    A_1 and A_2 hold the unit vectors e_r in rows r < R (other rows zero),
    so G_1 = G_2 = I, V = I and A_0 = M_0 V^-1 = M_0 exactly.  The nonzero
    at (i, r, r) has value x[i, r] and is the only one that reaches M_0(i, r)
    (the others, at (i, j, k) with j != k, multiply a zero).  Every column of
    x is an integer vector with squared norm 1024^2, so lambda_r = 1024 and
    A_0(i, r) = x[i, r] / 1024 exactly, in FP32 as well.  An odd integer in
    [256, 512) has nine significant bits, so it lies exactly halfway between
    two BF16 numbers: 257, 261, 321, 385 (last kept bit even) are ties that
    round down, 259, 263, 323, 387 ties that round up; a truncating store
    gets the latter wrong, a round-half-away-from-zero store the former."""
    rng = np.random.default_rng(seed)
    ties = [257, 259, 261, 263, 321, 323, 385, 387, 258]
    x = np.zeros((I0, R), np.int64)
    for r in range(R):
        vals = [int(v) * (1 if rng.random() < 0.5 else -1)
                for v in rng.choice(ties, size=6, replace=False)]
        rest = 1024 * 1024 - sum(v * v for v in vals)
        vals += [v * (1 if rng.random() < 0.5 else -1) for v in _sum_of_squares(rest)]
        rows = rng.choice(I0, size=len(vals), replace=False)
        x[rows, r] = vals
    ii, rr = np.nonzero(x)
    coords = [(int(i), int(r), int(r)) for i, r in zip(ii, rr)]
    vals = [float(x[i, r]) for i, r in zip(ii, rr)]
    seen = set(coords)
    while len(coords) < len(ii) + 1500:          # filler off the diagonal j == k
        c = (int(rng.integers(I0)), int(rng.integers(I1)), int(rng.integers(I2)))
        if c[1] != c[2] and c not in seen:
            seen.add(c)
            coords.append(c)
            vals.append(float(rng.integers(-8, 9)))
    order = rng.permutation(len(coords))
    idx = np.array(coords, np.int32)[order].T.copy()
    v = np.array(vals, np.float32)[order]
    a0 = rng.integers(-4, 5, (I0, R)).astype(np.float32) / 4
    a1 = np.zeros((I1, R), np.float32)
    a2 = np.zeros((I2, R), np.float32)
    a1[np.arange(R), np.arange(R)] = 1.0
    a2[np.arange(R), np.arange(R)] = 1.0
    return (I0, I1, I2), idx, v, [a0, a1, a2], x


def test_cp_als_bf16_store_is_round_to_nearest_even():
    """The BF16 store of the CP-ALS update rounds the FP64 result to nearest,
    ties to even (Alg. cp-als normalisation and store; BF16 reading of the
    precision form).  On the tensor above the first mode update is exact, so
    the stored bits must equal the library conversion (torch, CPU) of the
    oracle's FP64 values bit for bit."""
    dims, idx, v, facs0, x = _bf16_tie_tensor()
    R = facs0[0].shape[1]
    d = dev()
    p = Plan(torch.from_numpy(idx).to(d), torch.from_numpy(v).to(d), dims, R, g=64)
    facs = [torch.from_numpy(f).to(d).to(torch.bfloat16) for f in facs0]
    p.cp_als_sweep(facs)
    torch.cuda.synchronize()
    of, _, _, ridge, _ = oracle.cp_als_sweep(dims, idx, v, [f.astype(np.float64) for f in facs0])
    assert ridge == 0
    a0 = of[0]
    # the oracle's mode-0 update is the exact quotient x / 1024
    assert np.array_equal(a0, x / 1024.0)
    f32 = a0.astype(np.float32)
    assert np.array_equal(f32.astype(np.float64), a0)          # exact in FP32 too
    want = torch.from_numpy(f32).to(torch.bfloat16).view(torch.int16).numpy()
    got = facs[0].cpu().view(torch.int16).numpy()
    bad = np.argwhere(got != want)
    assert bad.size == 0, (f"{len(bad)} stored BF16 values differ from round-to-nearest-even; "
                           f"first at {tuple(bad[0])}: value {a0[tuple(bad[0])]!r}, "
                           f"bits {got[tuple(bad[0])] & 0xffff:#06x} vs {want[tuple(bad[0])] & 0xffff:#06x}")
    # the case has teeth: a truncating store and a round-half-away store
    # would each differ somewhere
    u = f32.view(np.uint32).astype(np.uint64)
    trunc = (u >> 16).astype(np.uint16)
    away = ((u + 0x8000) >> 16).astype(np.uint16)
    want16 = want.view(np.uint16)
    assert (trunc != want16).any() and (away != want16).any()
    ties = np.abs(x) % 2 == 1
    assert ties.sum() >= 32


def test_cp_als_gpu_converges_on_planted_tensor():
    rng = np.random.default_rng(5)
    dims, R = (12, 10, 8), 3
    true = [rng.standard_normal((d, R)) for d in dims]
    X = np.einsum("ir,jr,kr->ijk", *true)
    idx = np.array(np.unravel_index(np.arange(X.size), dims)).astype(np.int32)
    vals = X.reshape(-1).astype(np.float32)
    d = dev()
    p = Plan(torch.from_numpy(idx).to(d), torch.from_numpy(vals).to(d), dims, R, g=64)
    facs = [torch.from_numpy(rng.random((n, R)).astype(np.float32)).to(d) for n in dims]
    fit = None
    for _ in range(200):
        lam, fit = p.cp_als_sweep(facs)
    assert fit.item() > 1 - 1e-4, fit.item()


def test_profile_events_count_every_kernel_launch():
    """mttkrp_profile brackets each MTTKRP, remap, residual-MTTKRP and loss
    launch with HIP events; reads return one launch per mode per pass and
    reset what they returned."""
    dims, R = (60, 50, 40, 30), 16
    t = syn.random_tensor(dims, 4000, R, 77, zipf_s=1.1)
    p, facs = make_plan(t, g=64)
    N = len(dims)
    p.profile(True)
    p.mttkrp_all_modes(facs)
    p.cp_loss_grad(facs)                    # loss from the first residual pass
    p.cp_loss_grad(facs, grads=False)       # the loss pass alone
    torch.cuda.synchronize()
    for n in range(N):
        ms, c = p.profile_read(_abi.PROF_MTTKRP, n)
        assert c == 1 and ms > 0, (n, ms, c)
        ms, c = p.profile_read(_abi.PROF_RESID, n)
        assert c == 1 and ms > 0, (n, ms, c)
    ms, c = p.profile_read(_abi.PROF_LOSS)
    assert c == 1 and ms > 0
    ms, c = p.profile_read(_abi.PROF_REMAP)
    assert c == 2 * N and ms > 0          # one remap per pass of both sweeps
    for k in (_abi.PROF_MTTKRP, _abi.PROF_RESID, _abi.PROF_LOSS, _abi.PROF_REMAP):
        assert p.profile_read(k) == (0.0, 0)
    p.profile(False)
    p.mttkrp_all_modes(facs)
    torch.cuda.synchronize()
    assert p.profile_read(_abi.PROF_MTTKRP) == (0.0, 0)
    with pytest.raises(_abi.MttkrpError):
        p.profile_read(4)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("case", ALS_CASES[:3])
def test_cp_als_driver_equals_repeated_sweeps(case, dtype):
    """cp_als keeps the Gram matrices across sweeps instead of recomputing
    them; the Grams it keeps are those of the stored factors, so k sweeps of
    the driver are bit-identical to k calls of cp_als_sweep."""
    dims, nnz, R, seed, g = case
    say("als driver case", case, dtype)
    t = syn.random_tensor(dims, nnz, R, seed)
    idx, vals, f0 = to_dev(t, dtype)
    pa = Plan(idx, vals, dims, R, g=g)
    pb = Plan(idx, vals, dims, R, g=g)
    fa = [f.clone() for f in f0]
    fb = [f.clone() for f in f0]
    lam_a, fits = pa.cp_als(fa, max_sweeps=4, tol=0.0)
    assert fits.numel() == 4
    sweep_fits = []
    for _ in range(4):
        lam_b, fit_b = pb.cp_als_sweep(fb)
        sweep_fits.append(fit_b.item())
    torch.cuda.synchronize()
    for a, b in zip(fa, fb):
        assert torch.equal(a, b)
    assert torch.equal(lam_a, lam_b)
    assert fits.cpu().tolist() == sweep_fits
    # a tolerance above any fit change stops after two sweeps
    lam_c, fits_c = pa.cp_als([f.clone() for f in f0], max_sweeps=10, tol=2.0)
    assert fits_c.numel() == 2


def _dense_planted(dims, R, seed):
    rng = np.random.default_rng(seed)
    true = [rng.standard_normal((d, R)) for d in dims]
    idx = np.array(np.unravel_index(np.arange(int(np.prod(dims))), dims)).astype(np.int32)
    m = np.zeros(idx.shape[1])
    for r in range(R):
        term = np.ones(idx.shape[1])
        for n in range(len(dims)):
            term *= true[n][idx[n], r]
        m += term
    perm = rng.permutation(idx.shape[1])
    return idx[:, perm], m[perm].astype(np.float32), true


@pytest.mark.parametrize("dims,R,seed", [((30, 30, 30), 8, 1), ((20, 20, 20, 20), 8, 3)])
def test_cp_als_recovers_planted_dense_tensor(dims, R, seed):
    """A fully stored rank-R tensor: the driver converges to fit ~1 and the
    factor columns match the planted ones up to order and scale; the FP64
    oracle, looped from the same start, converges too."""
    idx, vals, true = _dense_planted(dims, R, seed)
    rng = np.random.default_rng(seed + 7)
    init = [rng.standard_normal((d, R)) for d in dims]
    d = dev()
    p = Plan(torch.from_numpy(idx).to(d), torch.from_numpy(vals).to(d), dims, R, g=256)
    facs = [torch.from_numpy(f.astype(np.float32)).to(d) for f in init]
    # fixed sweep count: near an exact fit the fit formula's cancellation
    # leaves noise of ~1e-4 in the fit, so a small tolerance is not a
    # usable stopping rule there; the factor match is the real check
    lam, fits = p.cp_als(facs, max_sweeps=150, tol=0.0)
    fits = fits.cpu().numpy()
    say("  sweeps", len(fits), "fit", fits[-1])
    assert len(fits) == 150
    assert fits[-1] > 1 - 1e-3, fits[-5:]
    for n in range(len(dims)):
        a = facs[n].cpu().numpy().astype(np.float64)
        a /= np.linalg.norm(a, axis=0)
        b = true[n] / np.linalg.norm(true[n], axis=0)
        cong = np.abs(a.T @ b).max(axis=0)          # best match of each planted column
        assert cong.min() > 0.9999, (n, cong.min())
    F = init
    for _ in range(150):
        F, _, ofit, _, _ = oracle.cp_als_sweep(dims, idx, vals, F)
    assert ofit > 1 - 1e-5


@pytest.mark.parametrize("case", LOSS_CASES[:3] + LOSS_CASES[4:])
def test_loss_and_gradient_bf16_factors(case):
    """BF16-stored factors: against the oracle on the BF16-rounded factors
    (accumulation error only) within the FP32 tolerance, and against the
    oracle on the FP32 factors (storage rounding included) within 2e-2."""
    dims, nnz, R, seed, g = case
    say("loss bf16 case", case)
    t = syn.random_tensor(dims, nnz, R, seed, factors="uniform")
    idx, vals, facs = to_dev(t, torch.bfloat16)
    p = Plan(idx, vals, dims, R, g=g)
    loss, grads = p.cp_loss_grad(facs)
    torch.cuda.synchronize()
    fb = [bf16_round(f) for f in t.factors]
    Lb, Gb = oracle.cp_loss_grad(dims, t.idx, t.vals, fb)
    assert abs(loss.item() - Lb) <= FP32_TOL * abs(Lb)
    refs = _grad_ref(t, fb)
    L32, G32 = oracle.cp_loss_grad(dims, t.idx, t.vals, [f.astype(np.float64) for f in t.factors])
    assert abs(loss.item() - L32) <= BF16_TOL * abs(L32)
    for k in range(len(dims)):
        gk = grads[k].cpu().numpy()
        check_close(gk, refs[k][0], refs[k][1], FP32_TOL, f"bf16 grad {k}")
        assert np.linalg.norm(gk - G32[k]) <= BF16_TOL * np.linalg.norm(G32[k])


def _random_loss_case(seed):
    """Randomly shaped small tensors for the residual kinds, which resolve
    the output row of every nonzero (2 to 6 modes, empty rows, shard sizes
    that are not multiples of 64, ranks for every lane form)."""
    rng = np.random.default_rng(2000 + seed)
    N = int(rng.choice([2, 3, 3, 4, 5, 6]))
    dims = tuple(int(rng.choice([1, 3, 37, 300, 2000, 50000])) for _ in range(N))
    if max(dims) == 1:
        dims = dims[:-1] + (60,)
    nnz = int(rng.integers(1, 3000))
    R = int(rng.choice([1, 4, 8, 16, 24, 32, 64]))
    g = int(rng.choice([1, 5, 63, 65, 200, 1024]))
    flags = int(rng.choice([0, _abi.FUSED_REMAP, _abi.UNPACKED_RECORDS]))
    return dims, nnz, R, g, flags


@pytest.mark.parametrize("seed", range(8))
def test_random_shapes_loss_gradient_and_bf16(seed):
    """On randomly shaped tensors: the loss and every gradient against the
    oracle (two routes), and BF16-stored factors' MTTKRP against the oracle
    on the BF16-rounded factors."""
    dims, nnz, R, g, flags = _random_loss_case(seed)
    say("random loss case", seed, dims, nnz, R, g, flags)
    t = syn.random_tensor(dims, nnz, R, 700 + seed, distinct=False, factors="uniform")
    idx, vals, facs = to_dev(t)
    p = Plan(idx, vals, dims, R, g=g, flags=flags)
    f64 = [f.astype(np.float64) for f in t.factors]
    L_ref, G_ref = oracle.cp_loss_grad(dims, t.idx, t.vals, f64)
    loss, grads = p.cp_loss_grad(facs)
    torch.cuda.synchronize()
    assert abs(loss.item() - L_ref) <= FP32_TOL * abs(L_ref), (loss.item(), L_ref)
    refs = _grad_ref(t, f64)
    for k in range(len(dims)):
        g_ = grads[k].cpu().numpy()
        assert np.linalg.norm(g_ - G_ref[k]) <= FP32_TOL * max(np.linalg.norm(G_ref[k]), 1e-30)
        check_close(g_, refs[k][0], refs[k][1], FP32_TOL, f"grad {k}")
    bf = [f.to(torch.bfloat16) for f in facs]
    outs = p.mttkrp_all_modes(bf)
    fb = [bf16_round(f) for f in t.factors]
    for n in range(len(dims)):
        ref, rabs = oracle.mttkrp(dims, t.idx, t.vals, fb, n, with_abs=True)
        check_close(outs[n].float().cpu().numpy(), ref, rabs, FP32_TOL, f"bf16 mode {n}")
