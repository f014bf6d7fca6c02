"""Pins for the FP64 oracle, against things other than itself.

Each check ties one oracle function to a closed form, a brute force on a
tiny input, exact integer arithmetic, or an invariant the paper states, so
that a dropped term, a wrong index or a transposed operand fails here.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2309_09131_amd import synthetic as syn


# ---------------------------------------------------------------- helpers
def dense_from_coo(dims, idx, vals):
    X = np.zeros(dims)
    np.add.at(X, tuple(idx.astype(np.int64)), vals.astype(np.float64))
    return X


def unfold(X, n):
    """Mode-n matricization (Sec. II-B): mode-n fibres as columns, the
    remaining modes swept with the earliest one varying fastest."""
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1, order="F")


def khatri_rao(mats):
    """Column-wise Kronecker product; the first matrix's index is slowest."""
    out = mats[0]
    for m in mats[1:]:
        out = (out[:, None, :] * m[None, :, :]).reshape(-1, m.shape[1])
    return out


def mttkrp_dense(X, factors, n):
    """X_(n) (A_{N-1} kr ... kr A_{n+1} kr A_{n-1} kr ... kr A_0)."""
    others = [factors[w] for w in reversed(range(X.ndim)) if w != n]
    return unfold(X, n) @ khatri_rao([np.asarray(f, np.float64) for f in others])


def mttkrp_einsum(X, factors, n):
    letters = "abcdefgh"[: X.ndim]
    terms = [letters] + [letters[w] + "z" for w in range(X.ndim) if w != n]
    spec = ",".join(terms) + "->" + letters[n] + "z"
    return np.einsum(spec, X, *[np.asarray(factors[w], np.float64)
                                for w in range(X.ndim) if w != n])


# ---------------------------------------------------------------- MTTKRP
@pytest.mark.parametrize("dims,R,dups", [
    ((5, 4, 3), 3, False), ((6, 5, 4), 7, True), ((3, 4, 2, 3), 5, False),
    ((3, 2, 4, 2, 3), 4, True), ((7, 6), 2, False)])
def test_mttkrp_matches_unfolding_khatri_rao_and_einsum(dims, R, dups):
    nnz = int(np.prod(dims)) // 2
    t = syn.random_tensor(dims, nnz, R, seed=11 + len(dims), distinct=not dups)
    X = dense_from_coo(dims, t.idx, t.vals)
    for n in range(len(dims)):
        got = oracle.mttkrp(dims, t.idx, t.vals, t.factors, n)
        ref1 = mttkrp_dense(X, t.factors, n)
        ref2 = mttkrp_einsum(X, t.factors, n)
        scale = np.abs(ref2).max()
        assert np.abs(got - ref1).max() <= 1e-14 * scale * 10
        assert np.abs(got - ref2).max() <= 1e-14 * scale * 10


def test_mttkrp_integer_inputs_are_exact():
    """Integer values and factors: the exact result is an integer; compare
    with int64 einsum (exact arithmetic, no rounding anywhere)."""
    dims = (9, 7, 5, 4)
    t = syn.random_tensor(dims, 600, 6, seed=3, distinct=False, int_values=True)
    Xi = np.zeros(dims, np.int64)
    np.add.at(Xi, tuple(t.idx.astype(np.int64)), t.vals.astype(np.int64))
    fi = [f.astype(np.int64) for f in t.factors]
    for n in range(4):
        got = oracle.mttkrp(dims, t.idx, t.vals, t.factors, n)
        letters = "abcd"
        spec = ",".join([letters] + [letters[w] + "z" for w in range(4) if w != n])
        ref = np.einsum(spec + "->" + letters[n] + "z", Xi,
                        *[fi[w] for w in range(4) if w != n])
        assert np.array_equal(got, ref.astype(np.float64))


def test_mttkrp_all_ones_factors_give_fibre_sums():
    dims = (30, 20, 10)
    t = syn.random_tensor(dims, 800, 4, seed=5)
    ones = [np.ones((d, 4), np.float32) for d in dims]
    for n in range(3):
        got = oracle.mttkrp(dims, t.idx, t.vals, ones, n)
        fib = np.bincount(t.idx[n], weights=t.vals.astype(np.float64),
                          minlength=dims[n])
        assert np.allclose(got, fib[:, None], rtol=1e-15, atol=0)


def test_mttkrp_rank_one_dense_closed_form():
    """X = a o b o c stored in full: M_0 = a * (b.b) * (c.c) per column."""
    rng = np.random.default_rng(1)
    a, b, c = rng.random(6), rng.random(5), rng.random(4)
    X = np.einsum("i,j,k->ijk", a, b, c)
    idx = np.array(list(itertools.product(range(6), range(5), range(4)))).T
    vals = X[tuple(idx)]
    fac = [np.stack([a, 2 * a], 1), np.stack([b, b], 1), np.stack([c, -c], 1)]
    got = oracle.mttkrp((6, 5, 4), idx, vals, fac, 0)
    ref0 = a * (b @ b) * (c @ c)
    assert np.allclose(got[:, 0], ref0, rtol=1e-14)
    assert np.allclose(got[:, 1], -ref0, rtol=1e-14)


def test_mttkrp_abs_scale_and_row_subset():
    dims = (40, 30, 20)
    t = syn.random_tensor(dims, 2000, 5, seed=8)
    t.vals = t.vals - 0.5                         # values of both signs
    full, fabs = oracle.mttkrp(dims, t.idx, t.vals, t.factors, 1, with_abs=True)
    X = dense_from_coo(dims, t.idx, t.vals)
    ref_abs = mttkrp_einsum(np.abs(X), [np.abs(f) for f in t.factors], 1)
    assert np.allclose(fabs, ref_abs, rtol=1e-13)
    rows = np.array([0, 7, 29, 3, 7, 0])          # rows may repeat
    sub, sabs = oracle.mttkrp_rows(dims, t.idx, t.vals, t.factors, 1, rows)
    assert np.allclose(sub, full[rows], rtol=1e-13, atol=1e-13)
    assert np.allclose(sabs, fabs[rows], rtol=1e-13)


# ---------------------------------------------------------------- layouts
def cyclic_lexsort(idx, n):
    """Order by (c_n, c_{n-1}, ..., c_{n+1}, input position)."""
    N, nnz = idx.shape
    keys = [np.arange(nnz)]                       # least significant first
    for k in range(N - 1, -1, -1):                # c_{n+1} ... c_n
        keys.append(idx[(n - k) % N])
    return np.lexsort(keys)


@pytest.mark.parametrize("dims,nnz,dups", [((7, 5, 6), 120, True),
                                            ((4, 6, 3, 5), 200, False),
                                            ((3, 2, 4, 2, 5), 150, True),
                                            ((9, 8), 40, True)])
def test_remap_replay_reaches_cyclic_lexicographic_layouts(dims, nnz, dups):
    t = syn.random_tensor(dims, nnz, 2, seed=21, distinct=not dups)
    N = len(dims)
    l0 = oracle.canonical_order(t.idx)
    assert np.array_equal(l0, cyclic_lexsort(t.idx, 0))
    layouts, perm, rps = oracle.remap_replay(dims, t.idx, l0)
    for n in range(N):
        assert np.array_equal(layouts[n], cyclic_lexsort(t.idx, n)), n
        # remap target is a bijection and moves slot i of L_n to perm[i]
        assert np.array_equal(np.sort(perm[n]), np.arange(nnz))
        nxt = np.empty(nnz, np.int64)
        nxt[perm[n]] = layouts[n]
        assert np.array_equal(nxt, layouts[n + 1])
        # row pointers are the prefix sums of the index histogram
        h = np.bincount(t.idx[n], minlength=dims[n])
        assert np.array_equal(rps[n], np.concatenate([[0], np.cumsum(h)]))
        # L_n is output-row contiguous and each row sits in its range
        c = t.idx[n][layouts[n]]
        assert np.all(np.diff(c) >= 0)
        for i in np.unique(c):
            assert np.all(c[rps[n][i]:rps[n][i + 1]] == i)
    # after N remaps the tensor is back in L_0 (one sweep is a cycle)
    assert np.array_equal(layouts[N], layouts[0])
    comp = np.arange(nnz)
    for n in range(N):
        comp = perm[n][comp]
    assert np.array_equal(comp, np.arange(nnz))


# ---------------------------------------------------------------- locality order
def z_curve(k):
    """The Z-order curve on a 2^k x 2^k grid by its recursive definition:
    the four quadrants in the order (a_hi, b_hi) = (0,0), (0,1), (1,0),
    (1,1), each traversed the same way (a is the more significant axis)."""
    if k == 0:
        return [(0, 0)]
    h = 1 << (k - 1)
    sub = z_curve(k - 1)
    return [(ah * h + a, bh * h + b) for ah in (0, 1) for bh in (0, 1) for a, b in sub]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_locality_order_follows_the_z_curve_on_full_grids(k):
    """One output row holding every point of a 2^k grid of its two leading
    inputs, in shuffled input order: the oracle's locality layout visits
    them along the Z curve.  Checked for output mode 0 of a 3-mode tensor
    (inputs c_2 then c_1) and output mode 1 of a 4-mode tensor (inputs c_0
    then c_3; c_2 is constant)."""
    s = 1 << k
    curve = z_curve(k)
    rng = np.random.default_rng(k)
    pts = np.array([(a, b) for a in range(s) for b in range(s)])
    pts = pts[rng.permutation(len(pts))]
    # 3 modes, output mode 0: c_{-1} = c_2 is the more significant input
    idx = np.stack([np.zeros(len(pts)), pts[:, 1], pts[:, 0]]).astype(np.int32)
    lay, _ = oracle.locality_layouts((1, s, s), idx)
    got = [(int(idx[2][e]), int(idx[1][e])) for e in lay[0]]
    assert got == curve
    # 4 modes, output mode 1: inputs c_0 (more significant) then c_3
    idx4 = np.stack([pts[:, 0], np.full(len(pts), 2), np.full(len(pts), 1),
                     pts[:, 1]]).astype(np.int32)
    lay4, _ = oracle.locality_layouts((s, 3, 2, s), idx4)
    got4 = [(int(idx4[0][e]), int(idx4[3][e])) for e in lay4[1]]
    assert got4 == curve


def spread_bits(x):
    """Bit k of a 32-bit value to bit 2k (mask-and-shift bit spreading)."""
    x = x.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    for sh, m in ((16, 0x0000FFFF0000FFFF), (8, 0x00FF00FF00FF00FF),
                  (4, 0x0F0F0F0F0F0F0F0F), (2, 0x3333333333333333),
                  (1, 0x5555555555555555)):
        x = (x | (x << np.uint64(sh))) & np.uint64(m)
    return x


def locality_lexsort(idx, n):
    """(c_n, Z(c_{n-1}, c_{n-2}), c_{n-3}, ..., c_{n+1}, input position)."""
    N, nnz = idx.shape
    keys = [np.arange(nnz)]                       # least significant first
    if N == 2:
        keys += [idx[(n - 1) % N], idx[n]]
        return np.lexsort(keys)
    for k in range(N - 1, 2, -1):                 # c_{n+1} ... c_{n-3}
        keys.append(idx[(n - k) % N])
    z = (spread_bits(idx[(n - 1) % N]) << np.uint64(1)) | spread_bits(idx[(n - 2) % N])
    keys += [z, idx[n]]
    return np.lexsort(keys)


@pytest.mark.parametrize("dims,nnz,dups", [((7, 5, 6), 120, True),
                                            ((40, 30, 20), 3000, False),
                                            ((4, 6, 3, 5), 200, False),
                                            ((3, 2, 4, 2, 5), 150, True),
                                            ((9, 8), 40, True),
                                            ((70000, 90000, 5000), 4000, False)])
def test_locality_layouts_invariants(dims, nnz, dups):
    t = syn.random_tensor(dims, nnz, 2, seed=23, distinct=not dups)
    N = len(dims)
    lay, perm = oracle.locality_layouts(dims, t.idx)
    _, _, rps = oracle.remap_replay(dims, t.idx)
    for n in range(N):
        assert np.array_equal(lay[n], locality_lexsort(t.idx, n)), n
        # output rows contiguous in the same ranges as the canonical layout
        c = t.idx[n][lay[n]]
        assert np.all(np.diff(c) >= 0)
        h = np.bincount(t.idx[n], minlength=dims[n])
        assert np.array_equal(rps[n], np.concatenate([[0], np.cumsum(h)]))
        # slot i of L_n goes to perm[i] of L_{n+1}
        assert np.array_equal(np.sort(perm[n]), np.arange(nnz))
        nxt = np.empty(nnz, np.int64)
        nxt[perm[n]] = lay[n]
        assert np.array_equal(nxt, lay[n + 1])
    assert np.array_equal(lay[N], lay[0])
    comp = np.arange(nnz)
    for n in range(N):
        comp = perm[n][comp]
    assert np.array_equal(comp, np.arange(nnz))
    if N == 2:                                    # one input: the canonical order
        for n in range(N):
            assert np.array_equal(lay[n], cyclic_lexsort(t.idx, n))


# ---------------------------------------------------------------- shards / LPT
def test_shard_tables_identities():
    t = syn.random_tensor((500, 40, 30), 6000, 2, seed=4, zipf_s=1.2)
    _, _, rps = oracle.remap_replay(t.dims, t.idx)
    for n, (m, g) in enumerate([(37, 64), (3, 50), (1, 1000)]):
        I = t.dims[n]
        sh = oracle.shards(I, rps[n], m, g)
        k = (I + m - 1) // m
        assert sh["ss_nnz"].sum() == t.nnz
        assert sh["start"].shape[0] == np.sum((sh["ss_nnz"] + g - 1) // g)
        assert np.all(sh["len"] >= 1) and np.all(sh["len"] <= g)
        # shards tile [0, nnz) in order and never cross a super-shard
        assert sh["start"][0] == 0
        assert np.array_equal(sh["start"][1:], (sh["start"] + sh["len"])[:-1])
        for s in range(sh["start"].shape[0]):
            j = sh["ss"][s]
            lo, hi = rps[n][j * m], rps[n][min((j + 1) * m, I)]
            assert lo <= sh["start"][s] and sh["start"][s] + sh["len"][s] <= hi
        assert sh["ss_nnz"].shape[0] == k


def test_lpt_graham_tight_example():
    """Two bins, jobs {3,3,2,2,2}: the greedy longest-first schedule has
    makespan 7 while the optimum is 6 = (3+3 | 2+2+2): the ratio is exactly
    4/3 - 1/(3*2), Graham's bound for the scheduling rule."""
    bins, load = oracle.lpt([3, 3, 2, 2, 2], 2)
    assert list(bins) == [0, 1, 0, 1, 0]
    assert sorted(load) == [5, 7]


def test_lpt_against_brute_force_optimum():
    rng = np.random.default_rng(7)
    for trial in range(60):
        k = int(rng.integers(1, 9))
        nu = int(rng.integers(1, 4))
        w = rng.integers(0, 12, k)
        bins, load = oracle.lpt(w, nu)
        # the bins really hold the assigned weights
        assert np.array_equal(np.bincount(bins, weights=w, minlength=nu)
                              .astype(np.int64), load)
        opt = min(max(np.bincount(a, weights=w, minlength=nu))
                  for a in itertools.product(range(nu), repeat=k))
        assert load.max() >= opt
        assert load.max() <= (4.0 / 3.0 - 1.0 / (3 * nu)) * opt + 1e-9
        # tie rules: heaviest first, lower id first; least loaded, lowest bin
        order = sorted(range(k), key=lambda j: (-w[j], j))
        ld = [0] * nu
        for j in order:
            b = min(range(nu), key=lambda i: (ld[i], i))
            assert bins[j] == b
            ld[b] += w[j]


# ---------------------------------------------------------------- CP-ALS
def _full_coo(X):
    idx = np.array(list(itertools.product(*[range(d) for d in X.shape]))).T
    return idx.astype(np.int32), X[tuple(idx)]


def _congruence(A, B):
    An = A / np.linalg.norm(A, axis=0)
    Bn = B / np.linalg.norm(B, axis=0)
    C = np.abs(An.T @ Bn)
    return min(max(C[i]) for i in range(C.shape[0]))


def test_cp_als_planted_exact_recovery_and_monotone_residual():
    rng = np.random.default_rng(2)
    dims, R = (12, 10, 8), 3
    # N(0,1) planted columns are well separated, so ALS converges in tens
    # of sweeps (all-positive columns swamp for hundreds)
    true = [rng.standard_normal((d, R)) for d in dims]
    X = np.einsum("ir,jr,kr->ijk", *true)
    idx, vals = _full_coo(X)
    fac = [rng.random((d, R)) for d in dims]
    xx = float(np.sum(X * X))
    prev = np.inf
    for sweep in range(1000):
        fac, lam, fit, ridge, res = oracle.cp_als_sweep(dims, idx, vals, fac)
        for r2 in res:                       # ALS never increases the error
            # (the residual formula cancels down to ~1e-16 * ||X||^2)
            assert r2 <= prev + 1e-13 * xx
            prev = r2
        Xh = np.einsum("r,ir,jr,kr->ijk", lam, *fac)
        rel = np.linalg.norm(Xh - X) / np.linalg.norm(X)
        if rel < 1e-10:
            break
    assert rel < 1e-10, (sweep, rel)
    # the reported fit is the explicit residual of the model
    assert abs((1 - fit) - rel) < 1e-7
    for n in range(3):
        assert _congruence(fac[n], true[n]) > 0.9999
        assert np.allclose(np.linalg.norm(fac[n], axis=0), 1.0)


def test_cp_als_zero_column_takes_the_ridge_and_matches_rank_minus_one():
    """A zero column r in the last factor makes every mode's V singular
    (row and column r of the Hadamard product vanish), so each mode update
    needs the ridge.  Column r stays zero with lambda_r = 0, and since the
    ridge is 1e-12 of the mean diagonal, the other columns, lambda and the
    fit equal the sweep of the same tensor at rank R - 1 without column r."""
    dims, R, r0 = (9, 8, 7), 4, 2
    t = syn.random_tensor(dims, 300, R, seed=12)
    fac = [np.array(f, np.float64) for f in t.factors]
    fac[2][:, r0] = 0.0
    got, lam, fit, ridge, _ = oracle.cp_als_sweep(dims, t.idx, t.vals, fac)
    keep = [r for r in range(R) if r != r0]
    ref, rlam, rfit, rridge, _ = oracle.cp_als_sweep(dims, t.idx, t.vals,
                                                     [f[:, keep] for f in fac])
    assert ridge == 3 and rridge == 0
    assert lam[r0] == 0.0
    for n in range(3):
        assert np.all(got[n][:, r0] == 0.0)
        assert np.allclose(got[n][:, keep], ref[n], rtol=1e-8, atol=1e-10)
    assert np.allclose(lam[keep], rlam, rtol=1e-8)
    assert abs(fit - rfit) < 1e-9


def test_cp_als_fit_matches_dense_residual_on_sparse_tensor():
    dims, R = (9, 8, 7, 6), 4
    t = syn.random_tensor(dims, 700, R, seed=9)
    X = dense_from_coo(dims, t.idx, t.vals)
    fac, lam, fit, ridge, res = oracle.cp_als_sweep(dims, t.idx, t.vals,
                                                   t.factors)
    Xh = np.einsum("r,ir,jr,kr,lr->ijkl", lam, *fac)
    resid = np.linalg.norm(X - Xh)
    assert abs((1 - fit) - resid / np.linalg.norm(X)) < 1e-10
    assert abs(res[-1] - resid ** 2) < 1e-8 * np.linalg.norm(X) ** 2
    # last mode update solves the normal equations: A V = M (before scaling)
    M = mttkrp_dense(X, [f for f in fac], 3)
    V = np.ones((R, R))
    for w in range(3):
        V *= fac[w].T @ fac[w]
    assert np.allclose((fac[3] * lam) @ V, M, rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------- loss
def test_loss_central_difference_is_exact():
    """m_e is affine in any single factor entry, so the loss is exactly
    quadratic in it and the central difference equals the derivative."""
    dims, R = (8, 7, 6), 5
    t = syn.random_tensor(dims, 150, R, seed=12, factors="uniform")
    L0, grads = oracle.cp_loss_grad(dims, t.idx, t.vals, t.factors)
    rng = np.random.default_rng(0)
    h = 1e-3
    for _ in range(64):
        k = int(rng.integers(0, 3))
        i = int(rng.choice(t.idx[k]))
        r = int(rng.integers(0, R))
        fp = [f.astype(np.float64).copy() for f in t.factors]
        fm = [f.astype(np.float64).copy() for f in t.factors]
        fp[k][i, r] += h
        fm[k][i, r] -= h
        Lp = oracle.cp_loss_grad(dims, t.idx, t.vals, fp, want_grad=False)
        Lm = oracle.cp_loss_grad(dims, t.idx, t.vals, fm, want_grad=False)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - grads[k][i, r]) <= 1e-9 * max(1.0, abs(fd)), (k, i, r)


def test_loss_against_dense_model_and_planted_truth():
    rng = np.random.default_rng(4)
    dims, R = (10, 9, 8), 3
    true = [rng.random((d, R)) for d in dims]
    X = np.einsum("ir,jr,kr->ijk", *true)
    t = syn.random_tensor(dims, 300, R, seed=13)
    vals = X[tuple(t.idx)]
    L, grads = oracle.cp_loss_grad(dims, t.idx, vals, true)
    assert L < 1e-25
    for g in grads:
        assert np.abs(g).max() < 1e-12
    # away from the truth: loss equals the masked dense residual
    other = [f + 0.1 for f in true]
    L2 = oracle.cp_loss_grad(dims, t.idx, vals, other, want_grad=False)
    Xo = np.einsum("ir,jr,kr->ijk", *other)
    assert np.isclose(L2, np.sum((vals - Xo[tuple(t.idx)]) ** 2), rtol=1e-13)


def test_loss_at_planted_truth_with_noise_matches_sigma():
    """With x = m + sigma*eps the expected loss at the truth is nnz*sigma^2."""
    rng = np.random.default_rng(6)
    dims, R, nnz = (60, 50, 40), 4, 20000
    true = [rng.random((d, R)) for d in dims]
    t = syn.random_tensor(dims, nnz, R, seed=14)
    m = np.einsum("er,er,er->e", *[true[n][t.idx[n]] for n in range(3)])
    sigma = 0.01 * np.sqrt(np.mean(m * m))
    vals = m + sigma * rng.standard_normal(nnz)
    L = oracle.cp_loss_grad(dims, t.idx, vals, true, want_grad=False)
    expect = nnz * sigma ** 2
    assert abs(L - expect) < 5 * np.sqrt(2.0 / nnz) * expect
