"""FP64 CP-ALS oracle (test infrastructure only).

The paper computes CPD by alternating least squares: the MTTKRP of Eq. (1) is
computed for each mode in turn, and the factors are normalised (Sec. II-A,
the CPD paragraph and the text after Eq. (1)).  It does not spell out the
least-squares solve, so this follows the textbook CP-ALS of the tensor survey
the paper cites (Kolda & Bader, "Tensor Decompositions and Applications"):

for each mode n in order:
    V   = Hadamard product of the Gram matrices G_m = A_m^T A_m, m != n
    M   = MTTKRP along mode n with the current factors
    A_n = M V^{-1}            (Cholesky factorisation V = L L^T, two triangular solves)
    lam = column 2-norms of A_n (a zero norm is replaced by 1);  A_n /= lam
    G_n = A_n^T A_n
after the last mode:
    <X, Xhat> = sum_r lam_r sum_i M[i, r] A_{N-1}[i, r]   (M of the last mode)
    |Xhat|^2  = lam^T (Hadamard product of all G_m) lam
    fit = 1 - sqrt(max(0, |X|^2 + |Xhat|^2 - 2 <X, Xhat>)) / |X|

|X|^2 is the sum of squared values after duplicate coordinates are merged.
A matrix V that is not positive definite raises ``numpy.linalg.LinAlgError``
(no silent regularisation).
"""

from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg

from . import ref


def coalesce(idx: np.ndarray, val: np.ndarray):
    """Merge duplicate coordinates by adding their values (FP64)."""
    idx = np.asarray(idx)
    if idx.shape[0] == 0:
        return idx.astype(np.uint32), np.zeros(0)
    u, inv = np.unique(idx, axis=0, return_inverse=True)
    v = np.zeros(u.shape[0], dtype=np.float64)
    np.add.at(v, inv.reshape(-1), np.asarray(val, dtype=np.float64))
    return u.astype(np.uint32), v


def gram(A: np.ndarray) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A


def hadamard_of_grams(G: Sequence[np.ndarray], skip: Optional[int] = None) -> np.ndarray:
    R = G[0].shape[0]
    V = np.ones((R, R), dtype=np.float64)
    for m, g in enumerate(G):
        if m != skip:
            V = V * g
    return V


def solve_mode(M: np.ndarray, V: np.ndarray) -> np.ndarray:
    """A = M V^{-1} through the Cholesky factor of V."""
    L = np.linalg.cholesky(V)
    Y = scipy.linalg.solve_triangular(L, np.asarray(M, dtype=np.float64).T, lower=True)
    X = scipy.linalg.solve_triangular(L.T, Y, lower=False)
    return X.T


def normalize_columns(A: np.ndarray):
    lam = np.sqrt(np.sum(np.asarray(A, dtype=np.float64) ** 2, axis=0))
    lam = np.where(lam == 0.0, 1.0, lam)
    return A / lam, lam


def fit_from_parts(normX2: float, M_last: np.ndarray, A_last: np.ndarray, lam: np.ndarray,
                   G: Sequence[np.ndarray]) -> float:
    inner = float(np.sum(lam * np.sum(M_last * A_last, axis=0)))
    xhat2 = float(lam @ hadamard_of_grams(G) @ lam)
    return 1.0 - np.sqrt(max(0.0, normX2 + xhat2 - 2.0 * inner)) / np.sqrt(normX2)


@dataclasses.dataclass
class AlsState:
    factors: List[np.ndarray]
    grams: List[np.ndarray]
    lam: np.ndarray
    normX2: float
    fits: List[float]
    iters: int = 0


def als_init(idx, val, dims, factors0) -> AlsState:
    A = [np.asarray(f, dtype=np.float64).copy() for f in factors0]
    R = A[0].shape[1]
    _, v = coalesce(idx, val)
    return AlsState(factors=A, grams=[gram(a) for a in A], lam=np.ones(R), normX2=float(np.sum(v * v)),
                    fits=[])


def als_iteration(state: AlsState, idx, val, dims, mttkrp_fn: Optional[Callable] = None,
                  on_mode: Optional[Callable] = None, threads: int = 1) -> float:
    """One sweep over all modes; returns the fit.  ``mttkrp_fn(n, factors)``
    defaults to the C oracle; ``on_mode(n, M, state)`` is called after each
    MTTKRP (before the update), for step-by-step comparisons."""
    N = len(dims)
    if mttkrp_fn is None:
        def mttkrp_fn(n, A):
            return ref.mttkrp(idx, val, dims, A, n, threads=threads)
    M = None
    for n in range(N):
        V = hadamard_of_grams(state.grams, skip=n)
        M = mttkrp_fn(n, state.factors)
        if on_mode is not None:
            on_mode(n, M, state)
        An = solve_mode(M, V)
        An, lam = normalize_columns(An)
        state.factors[n] = An
        state.grams[n] = gram(An)
        state.lam = lam
    fit = fit_from_parts(state.normX2, M, state.factors[N - 1], state.lam, state.grams)
    state.fits.append(fit)
    state.iters += 1
    return fit


def cp_als(idx, val, dims, factors0, n_iter: int, tol: Optional[float] = None, threads: int = 1
           ) -> AlsState:
    """Run ``n_iter`` sweeps, or stop early once |fit change| < ``tol``."""
    st = als_init(idx, val, dims, factors0)
    prev = None
    for _ in range(n_iter):
        f = als_iteration(st, idx, val, dims, threads=threads)
        if tol is not None and prev is not None and abs(f - prev) < tol:
            break
        prev = f
    return st
