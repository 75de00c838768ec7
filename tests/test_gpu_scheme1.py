"""Scheme 1 (Sec. III-B) on the GPU: layouts whose partitions hold whole
output rows dealt by LPT (MTTKRP_PART_ROWS_LPT) run the same partition kernel
with per-partition ranges and no carries.  Every mode against the FP64 oracle
(relative Frobenius <= 1e-5), including a row that holds most nonzeros,
empty tensors and rows, more partitions than rows, and 3-5 modes at R = 16,
32 and 64; and a CP-ALS sweep on a scheme-1 layout against the oracle's."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

LPT = capi.MTTKRP_PART_ROWS_LPT


def check_all_modes(t, R, kappa, seed=1):
    F = workloads.random_factors(t.dims, R, seed=seed)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, partitioner=LPT, lpt_parts=kappa))
    dF = gu.dev_factors(F)
    for n in range(len(t.dims)):
        got = gu.gpu_mttkrp(h, n, dF, R)
        assert np.all(np.isfinite(got)), f"mode {n}: unwritten output rows"
        ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, F, n)
        e = gu.rel_fro(got, ref)
        assert e <= 1e-5, f"mode {n}: rel err {e:.3e}"
        assert np.all(got[ref.sum(axis=1) == 0] == 0.0)
    h.free()


@pytest.mark.parametrize("dims,nnz,R,kappa,dist", [
    ((2000, 1500, 1000), 200_000, 32, 256, "zipf"),
    ((2000, 1500, 1000), 200_000, 16, 7, "zipf"),
    ((300, 250, 200, 40), 60_000, 64, 256, "zipf"),
    ((60, 50, 40, 30, 20), 30_000, 32, 100, "uniform"),
    ((5, 4000, 3000), 50_000, 32, 256, "uniform"),      # fewer rows than partitions in mode 0
    ((1000, 800, 600), 33, 16, 256, "uniform"),
    ((1000, 800, 600), 1, 64, 1, "uniform"),
])
def test_scheme1_matches_oracle(dims, nnz, R, kappa, dist):
    print("case scheme1", dims, nnz, R, kappa, dist, flush=True)
    t = workloads.random_tensor(dims, nnz, dist=dist, s=1.2 if dist == "zipf" else None, seed=5)
    check_all_modes(t, R, kappa)


def test_scheme1_one_row_holds_most_nonzeros():
    """Row 0 of mode 0 holds 90% of the nonzeros: one partition gets it whole."""
    print("case scheme1 heavy row", flush=True)
    rng = np.random.default_rng(9)
    nnz = 120_000
    idx = np.stack([np.where(rng.random(nnz) < 0.9, 0, rng.integers(0, 500, nnz)),
                    rng.integers(0, 700, nnz), rng.integers(0, 900, nnz)], axis=1).astype(np.uint32)
    val = rng.random(nnz).astype(np.float32)
    t = workloads.SparseTensor(idx=idx, val=val, dims=(500, 700, 900), nnz_requested=nnz)
    check_all_modes(t, 32, 64)


def test_scheme1_empty_tensor():
    t = workloads.SparseTensor(idx=np.zeros((0, 3), np.uint32), val=np.zeros(0, np.float32), dims=(10, 20, 30),
                               nnz_requested=0)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=16, partitioner=LPT, lpt_parts=8))
    dF = gu.dev_factors(workloads.random_factors(t.dims, 16, seed=1))
    for n in range(3):
        assert np.all(gu.gpu_mttkrp(h, n, dF, 16) == 0.0)
    h.free()


def test_scheme1_cp_als_sweep_vs_oracle():
    print("case scheme1 cp-als", flush=True)
    t = workloads.random_tensor((800, 600, 400), 60_000, dist="zipf", s=1.2, seed=11)
    R = 16
    F0 = workloads.random_factors(t.dims, R, seed=12)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, partitioner=LPT))
    dF = gu.dev_factors(F0)
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, dF, R)
    fits = []
    for _ in range(3):
        capi.cpd_als_iter(h, dF, lam, R, fit)
        fits.append(float(fit.item()))
    h.free()
    st = oracle.cp_als(t.idx, t.val, t.dims, F0, n_iter=3, threads=8)
    assert np.max(np.abs(np.array(fits) - np.array(st.fits))) <= 1e-6, (fits, st.fits)


def test_scheme1_refused_where_unsupported():
    t = workloads.random_tensor((100, 90, 80), 2000, seed=3)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=16, partitioner=LPT, lpt_parts=8))
    dF = gu.dev_factors(workloads.random_factors(t.dims, 16, seed=1))
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_batch_create([h], 16)
    assert e.value.status == capi.MTTKRP_EUNSUPPORTED
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_gather_probe(h, 0, dF, 16, 1)
    assert e.value.status == capi.MTTKRP_EUNSUPPORTED
    h.free()
