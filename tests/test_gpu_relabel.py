"""Degree-relabelled layouts (opts.relabel = 1) on the GPU: the MTTKRP with
factors in the new numbering equals the FP64 oracle on the original tensor
after the same renumbering of its rows, for fp32 and bf16 factors, device and
host builds, 3 and 4 modes; CP-ALS from renumbered starting factors follows
the oracle's fits."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,nnz,R,bf16,host", [
    ((3000, 2000, 1000), 200_000, 16, False, 0),
    ((3000, 2000, 1000), 200_000, 16, True, 0),
    ((70000, 500, 400), 150_001, 32, False, 1),
    ((400, 300, 200, 50), 100_000, 64, False, 0),
])
def test_relabelled_mttkrp_matches_oracle(dims, nnz, R, bf16, host):
    print("case relabel", dims, nnz, R, bf16, host, flush=True)
    t = workloads.random_tensor(dims, nnz, dist="zipf", s=1.2, seed=21)
    F = workloads.random_factors(t.dims, R, seed=22)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, relabel=1, build_on_host=host))
    perm = [capi.mttkrp_layout_perm(h, m) for m in range(len(dims))]
    Fnew = []
    for m, f in enumerate(F):
        g = np.empty_like(f)
        g[perm[m]] = f                                   # row perm[m][i] of the new factor is row i of the old
        Fnew.append(g)
    dF = gu.dev_factors(Fnew, dtype=torch.bfloat16 if bf16 else torch.float32)
    Fref = [oracle.bf16_round(f) for f in F] if bf16 else F
    for n in range(len(dims)):
        got = gu.gpu_mttkrp(h, n, dF, R, bf16=bf16)
        ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, Fref, n)
        e = gu.rel_fro(got[perm[n]], ref)                # output row perm[n][i] is original row i
        assert e <= 1e-5, f"mode {n}: rel err {e:.3e}"
    h.free()


def test_relabelled_cp_als_follows_oracle():
    print("case relabel cp-als", flush=True)
    R = 16
    t = workloads.random_tensor((500, 400, 300), 40_000, dist="zipf", s=1.2, seed=23)
    F0 = workloads.random_factors(t.dims, R, seed=24)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, relabel=1))
    perm = [capi.mttkrp_layout_perm(h, m) for m in range(3)]
    Fnew = []
    for m, f in enumerate(F0):
        g = np.empty_like(f)
        g[perm[m]] = f
        Fnew.append(g)
    d = gu.dev_factors(Fnew)
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, d, R)
    fits = []
    for _ in range(4):
        capi.cpd_als_iter(h, d, lam, R, fit)
        fits.append(float(fit.item()))
    st = oracle.cp_als(t.idx, t.val, t.dims, F0, n_iter=4, threads=8)
    assert max(abs(a - b) for a, b in zip(fits, st.fits)) <= 1e-5
    for m in range(3):
        got = d[m].cpu().numpy()[perm[m]]
        e = float(np.linalg.norm(got - st.factors[m]) / np.linalg.norm(st.factors[m]))
        assert e <= 1e-3, f"factor {m}: rel err {e:.2e}"
    h.free()
