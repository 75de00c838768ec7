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


def make_batch(count=12, seed=3, R=16, empty=True):
    rng = np.random.default_rng(seed)
    ts = []
    for i in range(count):
        dims = tuple(int(x) for x in rng.integers(100, 600, size=3))
        nnz = int(np.exp(rng.uniform(np.log(50), np.log(60_000))))
        if empty and i == count // 2:
            nnz = 0
        ts.append(workloads.random_tensor(dims, nnz, seed=1000 + i))
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R)) for t in ts]
    F = [workloads.random_factors(t.dims, R, seed=2000 + i) for i, t in enumerate(ts)]
    dF = [gu.dev_factors(f) for f in F]
    return ts, hs, F, dF


@pytest.mark.parametrize("R", [16, 32])
def test_batch_matches_oracle_and_single(R):
    print("case batch R", R, flush=True)
    ts, hs, F, dF = make_batch(R=R)
    b = capi.mttkrp_batch_create(hs, R)
    for n in range(3):
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
            assert gu.rel_fro(got, single) <= TOL
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
