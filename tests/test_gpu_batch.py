"""Batched MTTKRP (mttkrp_batch_run): every tensor of a batch against the FP64
oracle (relative Frobenius <= 1e-5) and against the single-tensor path; the
batch must repeat bit for bit and handle empty and tiny tensors."""

import numpy as np
import pytest
import torch

import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

TOL = 1e-5


def make_batch(count=12, seed=3, R=16, empty=True, nmodes=3, dist="uniform"):
    rng = np.random.default_rng(seed)
    ts = []
    for i in range(count):
        dims = tuple(int(x) for x in rng.integers(100, 600, size=nmodes))
        nnz = int(np.exp(rng.uniform(np.log(50), np.log(60_000))))
        if empty and i == count // 2:
            nnz = 0
        ts.append(workloads.random_tensor(dims, nnz, dist=dist, s=1.2 if dist == "zipf" else None, seed=1000 + i))
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R)) for t in ts]
    F = [workloads.random_factors(t.dims, R, seed=2000 + i) for i, t in enumerate(ts)]
    dF = [gu.dev_factors(f) for f in F]
    return ts, hs, F, dF


@pytest.mark.parametrize("nmodes,R,dist", [(3, 16, "uniform"), (3, 32, "uniform"), (3, 64, "zipf"),
                                           (4, 32, "zipf"), (5, 16, "uniform"), (5, 64, "zipf")])
def test_batch_matches_oracle_and_single(nmodes, R, dist):
    """Every mode count and rank the serving mix uses (3-5 modes, R = 16, 32,
    64), each batched instantiation against the oracle and bitwise against
    the single-tensor run."""
    print("case batch N", nmodes, "R", R, dist, flush=True)
    ts, hs, F, dF = make_batch(R=R, nmodes=nmodes, dist=dist)
    b = capi.mttkrp_batch_create(hs, R)
    for n in range(nmodes):
        outs = [torch.full((t.dims[n], R), float("nan"), device="cuda") for t in ts]
        capi.mttkrp_batch_run(b, n, dF, outs)
        torch.cuda.synchronize()
        for i, t in enumerate(ts):
            got = outs[i].cpu().numpy()
            assert np.all(np.isfinite(got)), f"tensor {i} mode {n}: unwritten output"
            ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, F[i], n)
            e = gu.rel_fro(got, ref)
            assert e <= TOL, f"tensor {i} mode {n}: rel err {e:.3e}"
            single = gu.gpu_mttkrp(hs[i], n, dF[i], R)
            assert np.array_equal(got.view(np.uint32), single.view(np.uint32)), \
                f"tensor {i} mode {n}: batched result differs from the single-tensor run"
    b.free()
    for h in hs:
        h.free()


def test_batch_repeatable_and_pointer_change():
    print("case batch repeat", flush=True)
    R = 16
    ts, hs, F, dF = make_batch(count=8, seed=5, R=R)
    b = capi.mttkrp_batch_create(hs, R, opts=dict(parts_per_cu=4))
    outs1 = [torch.empty((t.dims[1], R), device="cuda") for t in ts]
    outs2 = [torch.empty((t.dims[1], R), device="cuda") for t in ts]
    capi.mttkrp_batch_run(b, 1, dF, outs1)
    capi.mttkrp_batch_run(b, 1, dF, outs2)   # new output pointers: descriptors re-uploaded
    capi.mttkrp_batch_run(b, 1, dF, outs1)
    torch.cuda.synchronize()
    for a, c in zip(outs1, outs2):
        assert torch.equal(a, c)
    b.free()


def test_batch_errors():
    R = 16
    ts, hs, F, dF = make_batch(count=3, seed=7, R=R, empty=False)
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_batch_create(hs, 48)
    t4 = workloads.random_tensor((20, 30, 40, 50), 1000, seed=1)
    h4 = capi.mttkrp_layout_build(t4.idx, t4.val, t4.dims, opts=dict(max_R=R))
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_batch_create(hs + [h4], R)   # mixed N
    small = capi.mttkrp_layout_build(ts[0].idx, ts[0].val, ts[0].dims, opts=dict(max_R=16))
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_batch_create([small], 32)    # R above max_R


def test_batched_als_sweeps_equal_single():
    """Each tensor's CP-ALS sweeps give the same bits alone and in the batch."""
    print("case batch als", flush=True)
    R = 16
    ts, hs, F, _ = make_batch(count=6, seed=9, R=R, empty=False)
    b = capi.mttkrp_batch_create(hs, R)
    Fb = [gu.dev_factors(f) for f in F]
    Fs = [gu.dev_factors(f) for f in F]
    lam_b = [torch.zeros(R, dtype=torch.float64, device="cuda") for _ in ts]
    lam_s = [torch.zeros(R, dtype=torch.float64, device="cuda") for _ in ts]
    fit_b = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in ts]
    fit_s = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in ts]
    for i, h in enumerate(hs):
        capi.cpd_als_init(h, Fb[i], R)
    for _ in range(3):
        capi.cpd_als_batch_iter_async(b, Fb, lam_b, fit_b)
    torch.cuda.synchronize()
    out_b = [[f.clone() for f in fs] for fs in Fb]
    fits_b = [f.item() for f in fit_b]
    for i, h in enumerate(hs):
        capi.cpd_als_init(h, Fs[i], R)
        for _ in range(3):
            capi.cpd_als_iter_async(h, Fs[i], lam_s[i], R, fit_s[i])
        torch.cuda.synchronize()
        capi.cpd_als_status(h)
        for m in range(3):
            assert torch.equal(out_b[i][m], Fs[i][m]), f"tensor {i} factor {m}"
        assert fits_b[i] == fit_s[i].item()
        assert torch.equal(lam_b[i], lam_s[i])
    b.free()


def test_autotune_picks_a_candidate_and_keeps_results():
    """The autotuner returns one of its candidates, leaves it set on the
    layouts, and the batch built afterwards still matches the oracle and the
    single-tensor runs bit for bit."""
    print("case batch autotune", flush=True)
    R = 16
    ts, hs, F, dF = make_batch(count=10, seed=11, R=R)
    outs = [[torch.empty((d, R), device="cuda") for d in t.dims] for t in ts]
    best, times = capi.mttkrp_batch_autotune(hs, R, dF, outs, candidates=[1, 4, 16], reps=2)
    assert best in (1, 4, 16) and set(times) == {1, 4, 16} and all(v > 0 for v in times.values())
    assert all(capi.mttkrp_layout_info(h)["parts_per_cu"] == best for h in hs)
    b = capi.mttkrp_batch_create(hs, R)
    for n in range(3):
        o = [torch.empty((t.dims[n], R), device="cuda") for t in ts]
        capi.mttkrp_batch_run(b, n, dF, o)
        torch.cuda.synchronize()
        for i, t in enumerate(ts):
            got = o[i].cpu().numpy()
            assert gu.rel_fro(got, gu.oracle_mttkrp(t.idx, t.val, t.dims, F[i], n)) <= TOL
            assert np.array_equal(got.view(np.uint32), gu.gpu_mttkrp(hs[i], n, dF[i], R).view(np.uint32))
    b.free()
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_batch_autotune(hs, R, dF, outs, candidates=[0])
    for h in hs:
        h.free()


def test_batch256_workload_every_tensor():
    """The batching workload at its stated shape: 256 3-mode tensors, dims
    uniform in [100, 5000], nnz log-uniform in [1e3, 1e6] (35.3M nonzeros in
    all), R = 16, launched with the autotuned partition count.  Every output
    of every tensor and mode against the FP64 oracle (<= 1e-5 relative
    Frobenius per tensor and mode) and bitwise against its single-tensor
    run."""
    print("case batch256 full workload", flush=True)
    R = 16
    ts = workloads.batch_tensors(256)
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R)) for t in ts]
    F = [workloads.random_factors(t.dims, R, seed=3000 + i) for i, t in enumerate(ts)]
    dF = [gu.dev_factors(f) for f in F]
    outs = [[torch.empty((d, R), device="cuda") for d in t.dims] for t in ts]
    best, _ = capi.mttkrp_batch_autotune(hs, R, dF, outs, reps=2)
    print("  autotuned parts_per_cu", best, flush=True)
    b = capi.mttkrp_batch_create(hs, R)
    worst = 0.0
    for n in range(3):
        o = [torch.full((t.dims[n], R), float("nan"), device="cuda") for t in ts]
        capi.mttkrp_batch_run(b, n, dF, o)
        torch.cuda.synchronize()
        for i, t in enumerate(ts):
            got = o[i].cpu().numpy()
            e = gu.rel_fro(got, gu.oracle_mttkrp(t.idx, t.val, t.dims, F[i], n, threads=16))
            worst = max(worst, e)
            assert e <= TOL, f"tensor {i} mode {n}: rel err {e:.3e}"
            assert np.array_equal(got.view(np.uint32), gu.gpu_mttkrp(hs[i], n, dF[i], R).view(np.uint32)), \
                f"tensor {i} mode {n}: batched result differs from the single-tensor run"
    print(f"  worst rel fro {worst:.2e}", flush=True)
    b.free()
    for h in hs:
        h.free()


def test_bf16_batch_mttkrp_and_als_equal_single():
    """A batch created with factor_dtype BF16: the batched MTTKRP on bf16
    factors is bitwise mttkrp_run_bf16 of each tensor and matches the oracle
    fed the same bf16-rounded factors; batched CP-ALS sweeps of layouts built
    with bf16 factor copies are bitwise their single-tensor sweeps."""
    print("case batch bf16", flush=True)
    import oracle
    R = 32
    rng = np.random.default_rng(13)
    ts = []
    for i in range(6):
        dims = tuple(int(x) for x in rng.integers(100, 600, size=3))
        ts.append(workloads.random_tensor(dims, int(rng.integers(2000, 40000)), dist="zipf", s=1.2, seed=1300 + i))
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, factor_dtype=capi.MTTKRP_BF16))
          for t in ts]
    F = [workloads.random_factors(t.dims, R, seed=1400 + i) for i, t in enumerate(ts)]
    d16 = [gu.dev_factors(f, dtype=torch.bfloat16) for f in F]
    b = capi.mttkrp_batch_create(hs, R, opts=dict(factor_dtype=capi.MTTKRP_BF16))
    for n in range(3):
        outs = [torch.full((t.dims[n], R), float("nan"), device="cuda") for t in ts]
        capi.mttkrp_batch_run_bf16(b, n, d16, outs)
        torch.cuda.synchronize()
        for i, t in enumerate(ts):
            got = outs[i].cpu().numpy()
            assert np.array_equal(got.view(np.uint32), gu.gpu_mttkrp(hs[i], n, d16[i], R, bf16=True).view(np.uint32))
            ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, [oracle.bf16_round(f) for f in F[i]], n)
            assert gu.rel_fro(got, ref) <= TOL
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_batch_run(b, 0, [gu.dev_factors(f) for f in F], [torch.empty((t.dims[0], R), device="cuda")
                                                                      for t in ts])
    # batched CP-ALS on the bf16 copies against single sweeps
    Fb = [gu.dev_factors(f) for f in F]
    Fs = [gu.dev_factors(f) for f in F]
    lam_b = [torch.zeros(R, dtype=torch.float64, device="cuda") for _ in ts]
    lam_s = [torch.zeros(R, dtype=torch.float64, device="cuda") for _ in ts]
    fit_b = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in ts]
    fit_s = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in ts]
    for i, h in enumerate(hs):
        capi.cpd_als_init(h, Fb[i], R)
    for _ in range(3):
        capi.cpd_als_batch_iter_async(b, Fb, lam_b, fit_b)
    torch.cuda.synchronize()
    out_b = [[f.clone() for f in fs] for fs in Fb]
    fits_b = [f.item() for f in fit_b]
    for i, h in enumerate(hs):
        capi.cpd_als_init(h, Fs[i], R)
        for _ in range(3):
            capi.cpd_als_iter_async(h, Fs[i], lam_s[i], R, fit_s[i])
        torch.cuda.synchronize()
        capi.cpd_als_status(h)
        for m in range(3):
            assert torch.equal(out_b[i][m], Fs[i][m]), f"tensor {i} factor {m}"
        assert fits_b[i] == fit_s[i].item()
    b.free()
    # bf16 layouts in an fp32 batch: refused for CP-ALS
    b32 = capi.mttkrp_batch_create(hs, R)
    with pytest.raises(capi.MttkrpError):
        capi.cpd_als_batch_iter_async(b32, Fb, lam_b, fit_b)
    b32.free()
    for h in hs:
        h.free()
