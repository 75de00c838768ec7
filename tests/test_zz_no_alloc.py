"""mttkrp_run_noalloc (carry rows in the library's fixed per-device scratch
array, no allocation) against mttkrp_run on the same handle: bitwise equal
outputs on every mode, for two calls in a row with the second on a smaller
tensor (the array keeps the first call's contents), and both against the
FP64 oracle."""

import numpy as np
import pytest
import torch

import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _check(t, R, seed):
    F = workloads.random_factors(t.dims, R, seed=seed)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    dF = gu.dev_factors(F)
    plan = capi.mttkrp_launch_plan(t.nnz, len(t.dims), R)
    print(f"  nnz {t.nnz} R {R}: {plan['nparts']} partitions", flush=True)
    for n in range(len(t.dims)):
        ref = gu.gpu_mttkrp(h, n, dF, R)
        out = torch.full((t.dims[n], R), float("nan"), device="cuda")
        capi.mttkrp_run_noalloc(h, n, [None if m == n else dF[m] for m in range(len(t.dims))], out, R)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"mode {n}: differs from mttkrp_run"
        e = gu.rel_fro(got, gu.oracle_mttkrp(t.idx, t.val, t.dims, F, n))
        assert e <= 1e-5, f"mode {n}: rel err {e:.3e}"
    h.free()


def test_noalloc_matches_run_twice_second_smaller():
    print("case noalloc: large then small", flush=True)
    assert capi.mttkrp_noalloc_scratch_bytes() == 4 << 20
    big = workloads.random_tensor((4000, 3000, 2000), 2_000_000, dist="zipf", s=1.2, seed=41)
    small = workloads.random_tensor((500, 400, 300), 30_000, dist="zipf", s=1.2, seed=42)
    _check(big, 64, seed=43)
    _check(small, 32, seed=44)
