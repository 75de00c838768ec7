"""Hot-steps copies on the GPU (opts hot_steps=1: rows ordered by which of
their input rows are held in LDS, padded to whole wave steps, run by the step
kernel).  Every mode against the FP64 oracle (relative Frobenius <= 1e-5; bf16
factors against the oracle fed the same bf16-rounded factors), bitwise
repeatability, the no-allocation entry point, CP-ALS sweeps, the refusals,
and edge cases: one nonzero, a ragged 33, a mode shorter than the hot-row
count (every row hot), uniform indices (few hot rows), a row holding most of
the nonzeros, empty rows."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def steps_layout(t, R, dtype=capi.MTTKRP_FP32, **kw):
    return capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, hot_steps=1, factor_dtype=dtype, **kw))


def check_modes(t, R, dtype=capi.MTTKRP_FP32, seed=1, **kw):
    F = workloads.random_factors(t.dims, R, seed=seed)
    h = steps_layout(t, R, dtype, **kw)
    bf16 = dtype == capi.MTTKRP_BF16
    dF = gu.dev_factors(F, dtype=torch.bfloat16 if bf16 else torch.float32)
    Fref = [oracle.bf16_round(f) for f in F] if bf16 else F
    outs = []
    for n in range(len(t.dims)):
        got = gu.gpu_mttkrp(h, n, dF, R, bf16=bf16)
        assert np.all(np.isfinite(got)), f"mode {n}: unwritten output rows"
        ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, Fref, n)
        e = gu.rel_fro(got, ref)
        assert e <= 1e-5, f"mode {n}: rel err {e:.3e}"
        assert np.all(got[~np.any(ref != 0, axis=1)] == 0.0)
        again = gu.gpu_mttkrp(h, n, dF, R, bf16=bf16)
        assert np.array_equal(got.view(np.uint32), again.view(np.uint32)), f"mode {n}: not repeatable"
        outs.append(got)
    return h, dF, outs


@pytest.mark.parametrize("dims,nnz,R,dist", [
    ((4000, 3000, 2000), 1_000_000, 32, "zipf"),
    ((4000, 3000, 2000), 600_000, 16, "zipf"),
    ((4000, 3000, 2000), 600_000, 64, "zipf"),
    ((600, 500, 400, 60), 400_000, 32, "zipf"),
    ((600, 500, 400, 60), 200_000, 64, "zipf"),
    ((3000, 2500, 2000), 300_000, 32, "uniform"),
    ((50, 3000, 40), 100_000, 32, "zipf"),          # short modes: every row of them hot
    ((1000, 800, 600), 33, 32, "uniform"),
    ((1000, 800, 600), 1, 16, "uniform"),
])
def test_steps_match_oracle(dims, nnz, R, dist):
    print("case steps", dims, nnz, R, dist, flush=True)
    t = workloads.random_tensor(dims, nnz, dist=dist, s=1.2 if dist == "zipf" else None, seed=3)
    h, _, _ = check_modes(t, R)
    h.free()


@pytest.mark.parametrize("nmodes,R", [(3, 32), (3, 64), (4, 32)])
def test_steps_bf16_factors(nmodes, R):
    print("case steps bf16", nmodes, R, flush=True)
    dims = (3000, 2000, 1500) if nmodes == 3 else (600, 500, 400, 60)
    t = workloads.random_tensor(dims, 500_000, dist="zipf", s=1.2, seed=8)
    h, _, _ = check_modes(t, R, dtype=capi.MTTKRP_BF16)
    h.free()


def test_steps_heavy_row_and_partition_counts():
    """Row 0 of mode 0 holds 90% of the nonzeros (its steps span many waves and
    partitions); results agree across partition counts to rounding."""
    print("case steps heavy row", flush=True)
    rng = np.random.default_rng(9)
    nnz = 400_000
    idx = np.stack([np.where(rng.random(nnz) < 0.9, 0, rng.integers(0, 500, nnz)),
                    rng.integers(0, 700, nnz), rng.integers(0, 900, nnz)], axis=1).astype(np.uint32)
    idx = np.unique(idx, axis=0)
    t = workloads.SparseTensor(idx=idx, val=rng.random(idx.shape[0]).astype(np.float32), dims=(500, 700, 900),
                               nnz_requested=idx.shape[0])
    h1, dF, o1 = check_modes(t, 32, parts_per_cu=1)
    h8, _, o8 = check_modes(t, 32, parts_per_cu=16)
    for a, b in zip(o1, o8):
        assert gu.rel_fro(a, b) <= 1e-6
    h1.free()
    h8.free()


def test_steps_noalloc_and_cp_als():
    print("case steps noalloc + cp-als", flush=True)
    t = workloads.random_tensor((3000, 2000, 1000), 400_000, dist="zipf", s=1.2, seed=12)
    R = 32
    F0 = workloads.random_factors(t.dims, R, seed=13)
    h = steps_layout(t, R)
    dF = gu.dev_factors(F0)
    for n in range(3):
        ref = gu.gpu_mttkrp(h, n, dF, R)
        out = torch.full((t.dims[n], R), float("nan"), device="cuda")
        capi.mttkrp_run_noalloc(h, n, [None if m == n else dF[m] for m in range(3)], out, R)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, dF, R)
    fits = []
    for _ in range(3):
        capi.cpd_als_iter(h, dF, lam, R, fit)
        fits.append(float(fit.item()))
    h.free()
    st = oracle.cp_als(t.idx, t.val, t.dims, F0, n_iter=3, threads=8)
    print("  fits", fits, "oracle", st.fits, flush=True)
    assert np.max(np.abs(np.array(fits) - np.array(st.fits))) <= 1e-6


def test_steps_refusals():
    t = workloads.random_tensor((300, 200, 100), 20_000, dist="zipf", s=1.2, seed=2)
    h = steps_layout(t, 32)
    dF = gu.dev_factors(workloads.random_factors(t.dims, 32, seed=1))
    out = torch.empty((300, 16), device="cuda")
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_run(h, 0, [None] + [f[:, :16].contiguous() for f in dF[1:]], out, 16)
    assert e.value.status == capi.MTTKRP_EUNSUPPORTED
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_run_bf16(h, 0, [f.to(torch.bfloat16) for f in dF], torch.empty((300, 32), device="cuda"), 32)
    assert e.value.status == capi.MTTKRP_EUNSUPPORTED
    for call in (lambda: capi.mttkrp_batch_create([h], 32), lambda: capi.mttkrp_gather_probe(h, 0, dF, 32, 1),
                 lambda: capi.mttkrp_run_scheme2(h, 0, dF, torch.empty((300, 32), device="cuda"), 32)):
        with pytest.raises(capi.MttkrpError) as e:
            call()
        assert e.value.status == capi.MTTKRP_EUNSUPPORTED
    h.free()
    t5 = workloads.random_tensor((30, 20, 10, 8, 6), 2000, seed=2)
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_layout_build(t5.idx, t5.val, t5.dims, opts=dict(hot_steps=1))
    assert e.value.status == capi.MTTKRP_EUNSUPPORTED
