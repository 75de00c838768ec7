"""GPU CP-ALS sweeps (cpd_als_init / cpd_als_iter) against the FP64 oracle.

Each mode update solves the normal equations A_n V = M.  The check is
teacher-forced and independent of how well V is conditioned: for every mode,
in sweep order, the oracle computes M from the GPU's own factors at that
point of the sweep (updated factors for earlier modes, previous ones for
later modes) and V from their Gram matrices; the GPU's normalised A_n must
satisfy A_n diag(lam) V = M to FP32 accuracy for some column scaling lam,
and its columns must have unit norm.  The fit must equal the oracle's fit
formula evaluated on the GPU's factors.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def normal_eq_residual(A_new, V, M):
    """min over lam of |A diag(lam) V - M| / |M| (least squares in lam)."""
    I, R = A_new.shape
    # column r of A diag(lam) V = sum_k lam_k A[:, k] V[k, r]
    cols = np.stack([np.outer(A_new[:, k], V[k, :]).reshape(-1) for k in range(R)], axis=1)
    lam, *_ = np.linalg.lstsq(cols, M.reshape(-1), rcond=None)
    res = np.linalg.norm(cols @ lam - M.reshape(-1)) / np.linalg.norm(M)
    return float(res), lam


def run_sweeps(t, R, iters, dtype=capi.MTTKRP_FP32, seed=0, check=True, tol=2e-5):
    F0 = workloads.random_factors(t.dims, R, seed=seed)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, factor_dtype=dtype))
    dF = gu.dev_factors(F0)
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, dF, R)
    fits = []
    N = len(t.dims)
    val64 = t.val.astype(np.float64)
    for it in range(iters):
        before = [f.cpu().numpy().astype(np.float64) for f in dF]
        capi.cpd_als_iter(h, dF, lam, R, fit)
        torch.cuda.synchronize()
        after = [f.cpu().numpy().astype(np.float64) for f in dF]
        fits.append(float(fit.item()))
        if not check:
            continue
        cur = list(before)
        for n in range(N):
            use = cur
            if dtype == capi.MTTKRP_BF16:
                use = [oracle.bf16_round(c.astype(np.float32)).astype(np.float64) for c in cur]
            M = oracle.mttkrp(t.idx, val64, t.dims, use, n, threads=8)
            V = oracle.hadamard_of_grams([oracle.gram(c) for c in cur], skip=n)
            res, lam_fit = normal_eq_residual(after[n], V, M)
            assert res <= tol, f"iter {it} mode {n}: normal-equation residual {res:.3e}"
            norms = np.linalg.norm(after[n], axis=0)
            assert np.max(np.abs(norms - 1.0)) <= 1e-5, f"iter {it} mode {n}: column norms {norms}"
            cur[n] = after[n]
        # fit formula on the GPU's own factors
        lam_h = lam.cpu().numpy()
        M_last = oracle.mttkrp(t.idx, val64, t.dims, cur if dtype == capi.MTTKRP_FP32 else
                              [oracle.bf16_round(c.astype(np.float32)).astype(np.float64) for c in cur], N - 1,
                              threads=8)
        # lambda of the last mode: column norms of M V^{-1}, consistent with the normal equations
        st = oracle.als_init(t.idx, t.val, t.dims, cur)
        fit_ref = oracle.fit_from_parts(st.normX2, M_last, after[N - 1], lam_h, [oracle.gram(c) for c in cur])
        assert abs(fits[-1] - fit_ref) <= 1e-6, f"iter {it}: fit {fits[-1]} vs formula on GPU factors {fit_ref}"
        assert np.allclose(lam_fit, lam_h, rtol=1e-3), (lam_fit[:4], lam_h[:4])
    h.free()
    return fits


def test_sweeps_small_uniform():
    print("case als small uniform", flush=True)
    t = workloads.random_tensor((1000, 800, 600), 100_000, seed=1)
    fits = run_sweeps(t, 16, iters=3)
    assert all(b >= a - 1e-6 for a, b in zip(fits, fits[1:])), fits


@pytest.mark.parametrize("R", [32, 64])
def test_sweeps_zipf_4mode(R):
    print("case als zipf 4-mode R", R, flush=True)
    t = workloads.random_tensor((3000, 2000, 1500, 200), 200_000, dist="zipf", s=1.1, values="lognormal", seed=2)
    run_sweeps(t, R, iters=2)


def test_sweeps_bf16_factors():
    print("case als bf16", flush=True)
    t = workloads.random_tensor((2000, 1500, 1000), 150_000, dist="zipf", s=1.2, seed=3)
    run_sweeps(t, 32, iters=2, dtype=capi.MTTKRP_BF16)


def test_fit_trajectory_vs_oracle():
    """Same start, five sweeps on the 1000x800x600, 100k-nonzero tensor at R=16:
    the GPU (fp32 factors, FP64 normal equations) and the FP64 oracle fits agree
    within 1e-5 absolute and, since these fits are near 1e-4, 1e-6 relative."""
    print("case als trajectory", flush=True)
    t = workloads.random_tensor((1000, 800, 600), 100_000, seed=1)
    R = 16
    gpu = run_sweeps(t, R, iters=5, check=False)
    st = oracle.cp_als(t.idx, t.val, t.dims, workloads.random_factors(t.dims, R, seed=0), n_iter=5, threads=8)
    print("gpu fits", gpu)
    print("oracle fits", st.fits)
    diff = np.abs(np.array(gpu) - np.array(st.fits))
    print("max |dfit|", diff.max(), "relative", (diff / np.abs(st.fits)).max())
    assert diff.max() <= 1e-5
    assert (diff / np.abs(st.fits)).max() <= 1e-6


def test_not_spd_reported():
    print("case als not spd", flush=True)
    t = workloads.random_tensor((300, 200, 100), 5000, seed=4)
    R = 16
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    dF = [torch.rand((d, 1), device="cuda").repeat(1, R).contiguous() for d in t.dims]  # identical columns
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, dF, R)
    with pytest.raises(capi.MttkrpError) as e:
        capi.cpd_als_iter(h, dF, lam, R)
    assert e.value.status == capi.MTTKRP_ENOTSPD
    # a later good sweep works again on the same handle
    dF = gu.dev_factors(workloads.random_factors(t.dims, R, seed=5))
    capi.cpd_als_init(h, dF, R)
    capi.cpd_als_iter(h, dF, lam, R)
    h.free()


def test_iter_requires_init():
    t = workloads.random_tensor((100, 90, 80), 1000, seed=6)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=16))
    dF = gu.dev_factors(workloads.random_factors(t.dims, 16, seed=1))
    lam = torch.empty(16, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.MttkrpError) as e:
        capi.cpd_als_iter(h, dF, lam, 16)
    assert e.value.status == capi.MTTKRP_EINVAL
    h.free()
