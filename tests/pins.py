"""Independent checks ("pins") for an MTTKRP implementation.

Each pin takes the implementation under test as ``f(idx, val, dims, factors,
mode) -> ndarray`` and raises AssertionError when it disagrees with
something the mathematics fixes independently of it: a dense unfolding times
an explicit Khatri-Rao product, the closed form for rank-1 tensors, slice
sums, a scipy sparse-matrix product, a hand-worked example, and invariants.
The pins are applied to the FP64 oracle (which must pass them all) and to
copies of the oracle with a planted mistake (each must fail at least one).
"""

from __future__ import annotations

import json
import os

import numpy as np
import scipy.sparse

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_fro(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def rand_coo(rng, dims, nnz, dup=0):
    """Random COO with ``dup`` extra entries that repeat earlier coordinates."""
    idx = np.stack([rng.integers(0, d, size=nnz) for d in dims], axis=1)
    if dup:
        extra = idx[rng.integers(0, nnz, size=dup)]
        idx = np.concatenate([idx, extra], axis=0)
    val = rng.standard_normal(idx.shape[0])
    return idx.astype(np.uint32), val


def rand_factors(rng, dims, R):
    return [rng.standard_normal((d, R)) for d in dims]


# ----------------------------------------------------------------- dense reference pieces
def dense(idx, val, dims):
    X = np.zeros(dims, dtype=np.float64)
    np.add.at(X, tuple(np.asarray(idx, dtype=np.int64).T), val)
    return X


def cyclic_order(n, N):
    return [(n + j) % N for j in range(1, N)]


def unfold(X, n):
    """Mode-n unfolding; columns sweep the other modes in cyclic order
    n+1, ..., N-1, 0, ..., n-1 with the first of them varying slowest."""
    N = X.ndim
    return np.transpose(X, [n] + cyclic_order(n, N)).reshape(X.shape[n], -1)


def khatri_rao(mats):
    """Column-wise Kronecker product; the first matrix's row index varies slowest."""
    R = mats[0].shape[1]
    cols = []
    for r in range(R):
        v = np.ones(1)
        for M in mats:
            v = np.kron(v, M[:, r])
        cols.append(v)
    return np.stack(cols, axis=1)


# ----------------------------------------------------------------- pins
def pin_dense_khatri_rao(f, seed=0, tol=1e-13):
    """P1: X_(n) (KR of the other factors in cyclic order) for N = 3, 4, 5."""
    rng = np.random.default_rng(seed)
    for dims in [(5, 4, 3), (6, 2, 7), (3, 4, 2, 5), (2, 3, 3, 2, 3)]:
        idx, val = rand_coo(rng, dims, nnz=max(3, int(0.3 * np.prod(dims))), dup=4)
        R = 3
        A = rand_factors(rng, dims, R)
        X = dense(idx, val, dims)
        for n in range(len(dims)):
            ref = unfold(X, n) @ khatri_rao([A[m] for m in cyclic_order(n, len(dims))])
            got = f(idx, val, dims, A, n)
            assert got.shape == ref.shape, (dims, n, got.shape, ref.shape)
            e = rel_fro(got, ref)
            assert e <= tol, f"dense-KR pin: dims={dims} mode={n} rel={e:.3e}"


def pin_rank1_closed_form(f, seed=1, tol=1e-12):
    """P2: X = x0 o x1 o x2 (all entries stored) gives
    M_n[i, r] = x_n[i] * prod_{m != n} (x_m^T A_m)[r]."""
    rng = np.random.default_rng(seed)
    for dims in [(4, 3, 5), (3, 2, 2, 4)]:
        xs = [rng.uniform(0.5, 1.5, size=d) for d in dims]
        grid = np.stack(np.meshgrid(*[np.arange(d) for d in dims], indexing="ij"), axis=-1).reshape(-1, len(dims))
        val = np.ones(grid.shape[0])
        for m, x in enumerate(xs):
            val = val * x[grid[:, m]]
        R = 4
        A = rand_factors(rng, dims, R)
        for n in range(len(dims)):
            w = np.ones(R)
            for m in range(len(dims)):
                if m != n:
                    w = w * (xs[m] @ A[m])
            ref = np.outer(xs[n], w)
            e = rel_fro(f(grid.astype(np.uint32), val, dims, A, n), ref)
            assert e <= tol, f"rank-1 pin: dims={dims} mode={n} rel={e:.3e}"


def pin_slice_sums(f, seed=2, tol=1e-13):
    """P3: all-ones factors give the slice sums of the values in every column."""
    rng = np.random.default_rng(seed)
    dims = (7, 5, 6)
    idx, val = rand_coo(rng, dims, 60, dup=5)
    R = 3
    A = [np.ones((d, R)) for d in dims]
    for n in range(3):
        s = np.bincount(idx[:, n].astype(np.int64), weights=val, minlength=dims[n])
        ref = np.repeat(s[:, None], R, axis=1)
        e = rel_fro(f(idx, val, dims, A, n), ref)
        assert e <= tol, f"slice-sum pin: mode={n} rel={e:.3e}"


def pin_matrix_case(f, seed=3, tol=1e-13):
    """P4: for N = 2 the MTTKRP is a sparse matrix times a dense matrix:
    M_0 = X A_1 and M_1 = X^T A_0 (scipy.sparse)."""
    rng = np.random.default_rng(seed)
    dims = (9, 7)
    idx, val = rand_coo(rng, dims, 30, dup=3)
    R = 4
    A = rand_factors(rng, dims, R)
    X = scipy.sparse.coo_matrix((val, (idx[:, 0].astype(np.int64), idx[:, 1].astype(np.int64))), shape=dims).tocsr()
    assert rel_fro(f(idx, val, dims, A, 0), X @ A[1]) <= tol
    assert rel_fro(f(idx, val, dims, A, 1), X.T @ A[0]) <= tol


def pin_handworked(f, tol=0.0):
    """A 2x3x2 example worked by hand from the elementwise definition."""
    with open(os.path.join(GOLDEN, "handworked_3mode.json")) as fh:
        g = json.load(fh)
    idx = np.array(g["idx"], dtype=np.uint32)
    val = np.array(g["val"], dtype=np.float64)
    A = [np.array(a, dtype=np.float64) for a in g["factors"]]
    for n in range(3):
        got = f(idx, val, g["dims"], A, n)
        ref = np.array(g["expected"][n])
        assert np.max(np.abs(got - ref)) <= tol, f"hand-worked pin: mode {n}: {got} vs {ref}"


def pin_invariants(f, seed=4, tol=1e-12):
    """P5: permutation of the nonzeros, relabelling of indices, linearity in
    the values and in each factor, column separability, split duplicates."""
    rng = np.random.default_rng(seed)
    dims = (8, 6, 7, 5)
    N = len(dims)
    idx, val = rand_coo(rng, dims, 80, dup=6)
    R = 5
    A = rand_factors(rng, dims, R)
    for n in range(N):
        base = f(idx, val, dims, A, n)
        # order of the nonzeros does not matter
        p = rng.permutation(idx.shape[0])
        assert rel_fro(f(idx[p], val[p], dims, A, n), base) <= tol
        # relabel every mode: input factors' rows move with the labels, output rows permute
        perms = [rng.permutation(d) for d in dims]
        idx2 = np.stack([perms[m][idx[:, m]] for m in range(N)], axis=1).astype(np.uint32)
        A2 = []
        for m in range(N):
            B = np.empty_like(A[m])
            B[perms[m]] = A[m]
            A2.append(B)
        got = f(idx2, val, dims, A2, n)
        assert rel_fro(got[perms[n]], base) <= tol
        # linearity in the values
        v2 = rng.standard_normal(val.shape[0])
        lin = f(idx, 2.0 * val - 3.0 * v2, dims, A, n)
        assert rel_fro(lin, 2.0 * base - 3.0 * f(idx, v2, dims, A, n)) <= tol
        # linearity in each input factor
        for m in range(N):
            if m == n:
                continue
            Bm = rng.standard_normal(A[m].shape)
            Aa = list(A)
            Aa[m] = A[m] + 0.5 * Bm
            Ab = list(A)
            Ab[m] = Bm
            assert rel_fro(f(idx, val, dims, Aa, n), base + 0.5 * f(idx, val, dims, Ab, n)) <= tol
        # column r depends only on column r of the factors
        for r in range(R):
            Ar = [a[:, r:r + 1].copy() for a in A]
            assert rel_fro(f(idx, val, dims, Ar, n)[:, 0], base[:, r]) <= tol
        # one value split over two entries at the same coordinate
        k = 3
        idx3 = np.concatenate([idx, idx[k:k + 1]], axis=0)
        val3 = np.concatenate([val, [val[k] * (2.0 / 3.0)]])
        val3[k] = val[k] / 3.0
        assert rel_fro(f(idx3, val3, dims, A, n), base) <= tol
    # the output mode's factor is never read
    for n in range(N):
        Az = list(A)
        Az[n] = np.full_like(A[n], np.nan)
        assert np.all(np.isfinite(f(idx, val, dims, Az, n)))


def pin_large_dense_and_slices(f, seed=5, tol=1e-12):
    """P1 and P3 on tensors of 6,000 to 9,000 nonzeros (duplicates included), so
    that an implementation which switches strategy above a few thousand
    nonzeros (the oracle goes multi-threaded at 4,096) is pinned there too."""
    rng = np.random.default_rng(seed)
    for dims in [(20, 18, 16), (9, 8, 7, 6)]:
        nnz = 6000 if len(dims) == 3 else 2800
        idx, val = rand_coo(rng, dims, nnz=nnz, dup=3000)
        assert idx.shape[0] >= 5000
        R = 3
        A = rand_factors(rng, dims, R)
        X = dense(idx, val, dims)
        for n in range(len(dims)):
            ref = unfold(X, n) @ khatri_rao([A[m] for m in cyclic_order(n, len(dims))])
            e = rel_fro(f(idx, val, dims, A, n), ref)
            assert e <= tol, f"large dense-KR pin: dims={dims} mode={n} rel={e:.3e}"
            ones = [np.ones((d, R)) for d in dims]
            s = np.bincount(idx[:, n].astype(np.int64), weights=val, minlength=dims[n])
            e = rel_fro(f(idx, val, dims, ones, n), np.repeat(s[:, None], R, axis=1))
            assert e <= tol, f"large slice-sum pin: dims={dims} mode={n} rel={e:.3e}"


ALL_PINS = [pin_dense_khatri_rao, pin_rank1_closed_form, pin_slice_sums, pin_matrix_case, pin_handworked,
            pin_invariants, pin_large_dense_and_slices]
