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


def run_sweeps(t, R, iters, dtype=capi.MTTKRP_FP32, seed=0, check=True, tol=2e-5, als_solve=0):
    F0 = workloads.random_factors(t.dims, R, seed=seed)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, factor_dtype=dtype, als_solve=als_solve))
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


def _with_duplicates(t, frac, seed):
    """The tensor plus `frac` of its nonzeros again, each copy at the same
    coordinate with a fresh value, all shuffled: a COO list whose coordinates
    repeat, which the library must merge by adding (linearity of Eq. (1))."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(t.nnz, int(frac * t.nnz), replace=False)
    idx = np.concatenate([t.idx, t.idx[pick]])
    val = np.concatenate([t.val, rng.uniform(0.0, 1.0, pick.size).astype(np.float32)])
    perm = rng.permutation(idx.shape[0])
    return workloads.SparseTensor(idx=np.ascontiguousarray(idx[perm]), val=np.ascontiguousarray(val[perm]),
                                  dims=tuple(t.dims), nnz_requested=int(idx.shape[0]))


@pytest.mark.parametrize("build_on_host", [0, 1])
def test_fit_with_duplicate_coordinates_vs_oracle(build_on_host):
    """Repeated coordinates are one entry holding their sum, so |X|^2 (and the
    fit) must be taken after merging.  Same start, four sweeps: the GPU fits
    (device and host layout builds) against the FP64 oracle, which merges the
    duplicates before |X|^2, within 1e-6 absolute."""
    print("case als duplicates, host build", build_on_host, flush=True)
    base = workloads.random_tensor((700, 500, 300), 60_000, dist="zipf", s=1.2, seed=21)
    t = _with_duplicates(base, 0.3, seed=22)
    R = 16
    F0 = workloads.random_factors(t.dims, R, seed=23)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, build_on_host=build_on_host))
    dF = gu.dev_factors(F0)
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, dF, R)
    gpu = []
    for _ in range(4):
        capi.cpd_als_iter(h, dF, lam, R, fit)
        torch.cuda.synchronize()
        gpu.append(float(fit.item()))
    h.free()
    st = oracle.cp_als(t.idx, t.val, t.dims, F0, n_iter=4, threads=8)
    # the merged tensor's |X|^2 differs from the sum of squares of the raw list
    _, merged = oracle.coalesce(t.idx, t.val)
    raw = float(np.sum(t.val.astype(np.float64) ** 2))
    assert abs(float(np.sum(merged * merged)) - raw) > 1e-3 * raw
    print("gpu fits", gpu, "oracle fits", st.fits, flush=True)
    assert np.max(np.abs(np.array(gpu) - np.array(st.fits))) <= 1e-6


def test_ill_conditioned_normal_equations():
    """Nearly collinear factor columns make V = Hadamard of the Grams SPD but
    ill-conditioned (cond ~ 6e6 here).  The GPU update (FP64 sweep-operator
    inverse, FP32 store) must satisfy the normal equations of the first mode
    it updates, and agree with the oracle's Cholesky solve of the same M (the
    GPU's own FP32 MTTKRP, bitwise the one the sweep uses) to the accuracy the
    conditioning allows: |dA| / |A| <= cond(V) * 1e-14 + 1e-6.  Solving from
    the FP64 M instead would compare the MTTKRP's rounding amplified by
    cond(V), not the solve."""
    print("case als ill-conditioned V", flush=True)
    t = workloads.random_tensor((900, 700, 500), 50_000, seed=31)
    R = 16
    rng = np.random.default_rng(32)
    F0 = []
    for d in t.dims:
        base = rng.uniform(0.5, 1.0, (d, 1))
        F0.append((base + 1e-3 * rng.standard_normal((d, R))).astype(np.float32))
    F64 = [f.astype(np.float64) for f in F0]
    V = oracle.hadamard_of_grams([oracle.gram(f) for f in F64], skip=0)
    cond = float(np.linalg.cond(V))
    print(f"  cond(V) = {cond:.2e}", flush=True)
    assert 1e5 < cond < 1e11
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    dF = gu.dev_factors(F0)
    M = gu.gpu_mttkrp(h, 0, dF, R).astype(np.float64)
    M64 = oracle.mttkrp(t.idx, t.val.astype(np.float64), t.dims, F64, 0, threads=8)
    assert gu.rel_fro(M, M64) <= 1e-5
    A_ref, _ = oracle.normalize_columns(oracle.solve_mode(M, V))
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, dF, R)
    capi.cpd_als_iter(h, dF, lam, R)
    torch.cuda.synchronize()
    h.free()
    # mode 0 is updated first, from the starting factors of modes 1 and 2
    A0 = dF[0].cpu().numpy().astype(np.float64)
    res, _ = normal_eq_residual(A0, V, M)
    err = float(np.linalg.norm(A0 - A_ref) / np.linalg.norm(A_ref))
    print(f"  normal-equation residual {res:.2e}, |dA|/|A| vs Cholesky {err:.2e}", flush=True)
    assert res <= 2e-5
    assert err <= cond * 1e-14 + 1e-6


# ---- the opt-in Cholesky solve (opts.als_solve = 1) ----

@pytest.mark.parametrize("R", [16, 32, 64])
def test_cholesky_solve_sweeps_teacher_forced(R):
    """Cholesky factor and per-row substitution: every mode update satisfies
    the oracle's normal equations, unit column norms, the fit formula."""
    print("case als cholesky", R, flush=True)
    t = workloads.random_tensor((400, 300, 200, 60), 40_000, dist="zipf", s=1.2, seed=41)
    run_sweeps(t, R, iters=2, als_solve=1)


def test_cholesky_solve_trajectory_matches_oracle_and_default():
    print("case als cholesky trajectory", flush=True)
    t = workloads.random_tensor((1000, 800, 600), 100_000, seed=1)
    R = 16
    chol = run_sweeps(t, R, iters=5, check=False, als_solve=1)
    sweep = run_sweeps(t, R, iters=5, check=False, als_solve=0)
    st = oracle.cp_als(t.idx, t.val, t.dims, workloads.random_factors(t.dims, R, seed=0), n_iter=5, threads=8)
    assert np.max(np.abs(np.array(chol) - np.array(st.fits))) <= 1e-5
    assert np.max(np.abs(np.array(chol) - np.array(sweep))) <= 1e-6


def test_cholesky_solve_not_spd_reported():
    print("case als cholesky not spd", flush=True)
    t = workloads.random_tensor((300, 200, 100), 5000, seed=4)
    R = 16
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, als_solve=1))
    dF = [torch.rand((d, 1), device="cuda").repeat(1, R).contiguous() for d in t.dims]
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, dF, R)
    with pytest.raises(capi.MttkrpError) as e:
        capi.cpd_als_iter(h, dF, lam, R)
    assert e.value.status == capi.MTTKRP_ENOTSPD
    h.free()


def test_cholesky_solve_ill_conditioned_matches_oracle_solve():
    """cond(V) ~ 6e6: the substitution solve of the GPU's own M agrees with the
    oracle's Cholesky solve to cond(V) * 1e-14 + 1e-6."""
    print("case als cholesky ill-conditioned", flush=True)
    t = workloads.random_tensor((900, 700, 500), 50_000, seed=31)
    R = 16
    rng = np.random.default_rng(32)
    F0 = []
    for d in t.dims:
        base = rng.uniform(0.5, 1.0, (d, 1))
        F0.append((base + 1e-3 * rng.standard_normal((d, R))).astype(np.float32))
    F64 = [f.astype(np.float64) for f in F0]
    V = oracle.hadamard_of_grams([oracle.gram(f) for f in F64], skip=0)
    cond = float(np.linalg.cond(V))
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, als_solve=1))
    dF = gu.dev_factors(F0)
    M = gu.gpu_mttkrp(h, 0, dF, R).astype(np.float64)
    A_ref, _ = oracle.normalize_columns(oracle.solve_mode(M, V))
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, dF, R)
    capi.cpd_als_iter(h, dF, lam, R)
    torch.cuda.synchronize()
    h.free()
    A0 = dF[0].cpu().numpy().astype(np.float64)
    res, _ = normal_eq_residual(A0, V, M)
    err = float(np.linalg.norm(A0 - A_ref) / np.linalg.norm(A_ref))
    print(f"  cond {cond:.2e}, residual {res:.2e}, |dA|/|A| vs oracle {err:.2e}", flush=True)
    assert res <= 2e-5
    assert err <= cond * 1e-14 + 1e-6


def test_cholesky_solve_batch_bitwise_single():
    """Batched CP-ALS sweeps with the Cholesky solve are bitwise the single
    sweeps; a batch mixing the two solves is refused."""
    print("case als cholesky batch", flush=True)
    R = 32
    ts = [workloads.random_tensor((300 + 50 * i, 200, 150), 8000 + 3000 * i, seed=60 + i) for i in range(4)]
    F0 = [workloads.random_factors(t.dims, R, seed=70 + i) for i, t in enumerate(ts)]
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, als_solve=1)) for t in ts]
    dF = [gu.dev_factors(f) for f in F0]
    lam = [torch.empty(R, dtype=torch.float64, device="cuda") for _ in ts]
    fit = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in ts]
    for h, d in zip(hs, dF):
        capi.cpd_als_init(h, d, R)
    b = capi.mttkrp_batch_create(hs, R)
    for _ in range(2):
        capi.cpd_als_batch_iter_async(b, dF, lam, fit)
    torch.cuda.synchronize()
    b.free()
    for i, (t, h) in enumerate(zip(ts, hs)):
        d = gu.dev_factors(F0[i])
        l1 = torch.empty(R, dtype=torch.float64, device="cuda")
        f1 = torch.empty(1, dtype=torch.float64, device="cuda")
        capi.cpd_als_init(h, d, R)
        for _ in range(2):
            capi.cpd_als_iter(h, d, l1, R, f1)
        assert float(f1.item()) == float(fit[i].item()), i
        for a, c in zip(d, dF[i]):
            assert torch.equal(a, c), i
    plain = capi.mttkrp_layout_build(ts[0].idx, ts[0].val, ts[0].dims, opts=dict(max_R=R))
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_batch_create([hs[0], plain], R)
    plain.free()
    for h in hs:
        h.free()
