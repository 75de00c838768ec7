"""16-bit input coordinates (copies whose input dimensions are all <= 65536):
every mode against the FP64 oracle and bitwise against the same layout with
32-bit coordinates (the arithmetic and order are the same), for 3-5 modes,
R = 16/32/64, fp32 and bf16 factors, host and device builds, a mix of 16-
and 32-bit copies in one tensor, dimensions of exactly 65536, ragged sizes,
and a batch of 16-bit tensors."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,nnz,R,bf16,host", [
    ((4000, 3000, 2000), 300_000, 32, False, 0),
    ((70000, 500, 400), 200_000, 16, False, 0),          # copy 0 16-bit, copies 1 and 2 32-bit
    ((65536, 65536, 300), 200_000, 64, False, 1),        # the largest 16-bit dimension, host build
    ((300, 250, 200, 40), 100_000, 32, True, 0),
    ((60, 50, 40, 30, 20), 50_000, 16, False, 1),
    ((500, 400, 300), 33, 32, False, 0),
])
def test_idx16_matches_wide_and_oracle(dims, nnz, R, bf16, host):
    print("case idx16", dims, nnz, R, bf16, host, flush=True)
    t = workloads.random_tensor(dims, nnz, dist="zipf", s=1.2, seed=6)
    F = workloads.random_factors(t.dims, R, seed=7)
    h16 = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, build_on_host=host))
    h32 = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, build_on_host=host, wide_indices=1))
    mask = capi.mttkrp_layout_info(h16)["idx16_modes"]
    want = sum(1 << n for n in range(len(dims)) if all(dims[m] <= 65536 for m in range(len(dims)) if m != n))
    assert mask == want and capi.mttkrp_layout_info(h32)["idx16_modes"] == 0
    dF = gu.dev_factors(F, dtype=torch.bfloat16 if bf16 else torch.float32)
    Fref = [oracle.bf16_round(f) for f in F] if bf16 else F
    for n in range(len(dims)):
        a = gu.gpu_mttkrp(h16, n, dF, R, bf16=bf16)
        b = gu.gpu_mttkrp(h32, n, dF, R, bf16=bf16)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"mode {n}: 16-bit and 32-bit copies differ"
        e = gu.rel_fro(a, gu.oracle_mttkrp(t.idx, t.val, t.dims, Fref, n))
        assert e <= 1e-5, f"mode {n}: rel err {e:.3e}"
    h16.free()
    h32.free()


def test_idx16_batch_and_cp_als():
    """A batch of 16-bit tensors: bitwise the single-tensor runs, and CP-ALS
    sweeps bitwise those of 32-bit copies."""
    print("case idx16 batch", flush=True)
    R = 16
    ts = [workloads.random_tensor((int(d0), 300, 200), 20_000 + 5000 * i, seed=40 + i)
          for i, d0 in enumerate([100, 700, 5000, 65536])]
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R)) for t in ts]
    assert all(capi.mttkrp_layout_info(h)["idx16_modes"] == 0b111 for h in hs)
    F = [workloads.random_factors(t.dims, R, seed=50 + i) for i, t in enumerate(ts)]
    dF = [gu.dev_factors(f) for f in F]
    b = capi.mttkrp_batch_create(hs, R)
    for n in range(3):
        outs = [torch.full((t.dims[n], R), float("nan"), device="cuda") for t in ts]
        capi.mttkrp_batch_run(b, n, dF, outs)
        torch.cuda.synchronize()
        for i, t in enumerate(ts):
            got = outs[i].cpu().numpy()
            assert np.array_equal(got.view(np.uint32), gu.gpu_mttkrp(hs[i], n, dF[i], R).view(np.uint32))
            assert gu.rel_fro(got, gu.oracle_mttkrp(t.idx, t.val, t.dims, F[i], n)) <= 1e-5
    b.free()
    t = ts[1]
    fits = []
    for wide in (0, 1):
        h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, wide_indices=wide))
        d = gu.dev_factors(F[1])
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
        fit = torch.empty(1, dtype=torch.float64, device="cuda")
        capi.cpd_als_init(h, d, R)
        for _ in range(2):
            capi.cpd_als_iter(h, d, lam, R, fit)
        fits.append((float(fit.item()), [x.cpu().numpy() for x in d]))
        h.free()
    assert fits[0][0] == fits[1][0]
    for a, c in zip(fits[0][1], fits[1][1]):
        assert np.array_equal(a.view(np.uint32), c.view(np.uint32))
    for h in hs:
        h.free()
