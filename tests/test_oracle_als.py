"""FP64 CP-ALS oracle against what the mathematics fixes (no GPU).

* every mode update is an exact least-squares solve, so the fit never drops;
* the fit computed from (M, Grams, lambda) equals 1 - |X - Xhat| / |X| with
  Xhat rebuilt densely from the factors;
* a tensor that is exactly sparse and of rank R is recovered (fit ~ 1 and the
  factors match after permutation and scaling);
* planted mistakes in the update (applied to the oracle module on the CPU
  through monkeypatch) break at least one of these checks.
"""

import itertools

import numpy as np
import pytest

import oracle
import oracle.als as als
from tests import pins


def dense_reconstruction(factors, lam):
    N = len(factors)
    R = lam.shape[0]
    dims = [f.shape[0] for f in factors]
    X = np.zeros(dims)
    for r in range(R):
        t = np.array(lam[r])
        for m in range(N):
            t = np.multiply.outer(t, factors[m][:, r])
        X += t
    return X


def random_problem(seed, dims=(9, 8, 7), nnz=150, R=4):
    rng = np.random.default_rng(seed)
    idx, _ = pins.rand_coo(rng, dims, nnz)
    idx, _ = als.coalesce(idx, np.ones(idx.shape[0]))
    val = rng.uniform(0.0, 1.0, idx.shape[0])
    A0 = [rng.uniform(0.0, 1.0, (d, R)) for d in dims]
    return idx, val, dims, A0


@pytest.mark.parametrize("dims", [(9, 8, 7), (6, 5, 4, 3)])
def test_fit_is_monotone(dims):
    idx, val, dims, A0 = random_problem(0, dims=dims, nnz=120)
    st = oracle.cp_als(idx, val, dims, A0, n_iter=25)
    f = np.array(st.fits)
    assert np.all(np.diff(f) >= -1e-12), f


def test_fit_formula_equals_dense_residual():
    idx, val, dims, A0 = random_problem(1)
    st = oracle.als_init(idx, val, dims, A0)
    X = pins.dense(idx, val, dims)
    for _ in range(4):
        fit = oracle.als_iteration(st, idx, val, dims)
        Xh = dense_reconstruction(st.factors, st.lam)
        fit_dense = 1.0 - np.linalg.norm(X - Xh) / np.linalg.norm(X)
        assert abs(fit - fit_dense) <= 1e-10, (fit, fit_dense)


def test_fit_with_duplicate_coordinates_equals_dense_residual():
    """Duplicate coordinates are one entry of X holding their sum (linearity of
    the elementwise definition), so |X|^2 must be taken after merging them.
    X is built densely with np.add.at, independently of the oracle's merge;
    the fit after each sweep must equal 1 - |X - Xhat| / |X| on it."""
    rng = np.random.default_rng(12)
    dims = (9, 8, 7)
    idx, val = pins.rand_coo(rng, dims, 120, dup=60)
    val = np.abs(val) + 0.1
    A0 = [rng.uniform(0.0, 1.0, (d, 4)) for d in dims]
    X = pins.dense(idx, val, dims)
    assert abs(np.sum(X * X) - np.sum(val * val)) > 1.0   # the merge matters here
    st = oracle.als_init(idx, val, dims, A0)
    assert abs(st.normX2 - float(np.sum(X * X))) <= 1e-12 * float(np.sum(X * X))
    for _ in range(3):
        fit = oracle.als_iteration(st, idx, val, dims)
        Xh = dense_reconstruction(st.factors, st.lam)
        fit_dense = 1.0 - np.linalg.norm(X - Xh) / np.linalg.norm(X)
        assert abs(fit - fit_dense) <= 1e-10, (fit, fit_dense)


def test_solve_mode_is_least_squares_solution():
    """A_n = M V^{-1} is the normal-equation solution: compare with lstsq on
    the explicit Khatri-Rao system (tiny dense case)."""
    rng = np.random.default_rng(2)
    dims = (5, 4, 3)
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((d, 3)) for d in dims]
    n = 0
    KR = pins.khatri_rao([A[m] for m in pins.cyclic_order(n, 3)])
    Xn = pins.unfold(X, n)
    ref = np.linalg.lstsq(KR, Xn.T, rcond=None)[0].T
    M = Xn @ KR
    V = oracle.hadamard_of_grams([oracle.gram(a) for a in A], skip=n)
    assert pins.rel_fro(oracle.solve_mode(M, V), ref) <= 1e-10


def test_not_spd_raises():
    M = np.ones((3, 2))
    V = np.array([[1.0, 1.0], [1.0, 1.0]])  # singular
    with pytest.raises(np.linalg.LinAlgError):
        oracle.solve_mode(M, V)


def planted_sparse_rank_r(seed, dims, R, density=0.3):
    rng = np.random.default_rng(seed)
    F = []
    for d in dims:
        A = np.zeros((d, R))
        for r in range(R):
            k = max(2, int(round(density * d)))
            rows = rng.choice(d, size=k, replace=False)
            A[rows, r] = rng.uniform(0.5, 1.0, size=k)
        F.append(A)
    X = dense_reconstruction(F, np.ones(R))
    nzc = np.argwhere(X != 0.0)
    return nzc.astype(np.uint32), X[tuple(nzc.T)], F


def factor_match_score(F_true, F_est):
    R = F_true[0].shape[1]
    nt = [f / np.linalg.norm(f, axis=0) for f in F_true]
    ne = [f / np.linalg.norm(f, axis=0) for f in F_est]
    best = 0.0
    for perm in itertools.permutations(range(R)):
        s = 0.0
        for r in range(R):
            t = 1.0
            for m in range(len(F_true)):
                t *= abs(float(nt[m][:, r] @ ne[m][:, perm[r]]))
            s += t
        best = max(best, s / R)
    return best


def run_recovery(seeds=range(5), iters=200):
    dims, R = (14, 12, 10), 3
    idx, val, F = planted_sparse_rank_r(11, dims, R)
    best_fit, best_fms = -np.inf, 0.0
    for s in seeds:
        rng = np.random.default_rng(100 + s)
        A0 = [rng.uniform(0.0, 1.0, (d, R)) for d in dims]
        st = oracle.cp_als(idx, val, dims, A0, n_iter=iters, tol=1e-12)
        if st.fits[-1] > best_fit:
            best_fit = st.fits[-1]
            best_fms = factor_match_score(F, st.factors)
    return best_fit, best_fms


def test_planted_recovery():
    fit, fms = run_recovery()
    assert fit >= 0.999, fit
    assert fms >= 0.99, fms


# ------------------------------------------------------------------ planted mistakes
def _check_all():
    """Run the three ALS checks; return the names of those that fail."""
    failed = []
    try:
        test_fit_is_monotone((9, 8, 7))
    except (AssertionError, np.linalg.LinAlgError):
        failed.append("monotone")
    try:
        test_fit_formula_equals_dense_residual()
    except (AssertionError, np.linalg.LinAlgError):
        failed.append("dense-residual")
    try:
        test_fit_with_duplicate_coordinates_equals_dense_residual()
    except (AssertionError, np.linalg.LinAlgError):
        failed.append("duplicates")
    try:
        fit, fms = run_recovery(seeds=range(2), iters=60)
        assert fit >= 0.99 and fms >= 0.95
    except (AssertionError, np.linalg.LinAlgError):
        failed.append("recovery")
    return failed


def test_checks_pass_for_correct_oracle():
    assert _check_all() == []


@pytest.mark.parametrize("kind", ["own_gram_in_V", "no_inverse", "lam_not_squared_out", "stale_gram",
                                  "inner_sign", "no_merge"])
def test_checks_catch_planted_als_mistake(kind, monkeypatch):
    if kind == "own_gram_in_V":
        orig = als.hadamard_of_grams
        monkeypatch.setattr(als, "hadamard_of_grams", lambda G, skip=None: orig(G, None))
    elif kind == "no_inverse":
        monkeypatch.setattr(als, "solve_mode", lambda M, V: np.asarray(M) @ V)
    elif kind == "lam_not_squared_out":
        orig = als.normalize_columns
        monkeypatch.setattr(als, "normalize_columns", lambda A: (orig(A)[0], np.sqrt(orig(A)[1])))
    elif kind == "stale_gram":
        monkeypatch.setattr(als, "gram", lambda A: np.eye(np.asarray(A).shape[1]) * 0 + np.asarray(A)[:1].T @ np.asarray(A)[:1] + np.eye(np.asarray(A).shape[1]))
    elif kind == "no_merge":
        # |X|^2 as the sum of the squared entries as given, duplicates not merged
        monkeypatch.setattr(als, "coalesce", lambda idx, val: (np.asarray(idx), np.asarray(val, dtype=np.float64)))
    elif kind == "inner_sign":
        orig = als.fit_from_parts
        monkeypatch.setattr(als, "fit_from_parts",
                            lambda nx, M, A, lam, G: orig(nx, -M, A, lam, G))
    assert _check_all(), f"planted ALS mistake {kind!r} not caught"
