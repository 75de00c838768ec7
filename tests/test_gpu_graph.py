"""CP-ALS sweeps and batched MTTKRPs captured into a HIP graph (through
torch.cuda.graph) must reproduce the eager results bit for bit, on every
replay, with eager work and synchronisations between the replays."""

import numpy as np
import pytest
import torch

import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_als_sweeps_in_graph_match_eager():
    print("case graph als", flush=True)
    R = 16
    K = 4
    t = workloads.random_tensor((800, 600, 500), 60_000, dist="zipf", s=1.2, seed=21)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    F0 = gu.dev_factors(workloads.random_factors(t.dims, R, seed=21))
    F = [f.clone() for f in F0]
    lam = torch.zeros(R, dtype=torch.float64, device="cuda")
    fit = torch.zeros(1, dtype=torch.float64, device="cuda")

    def reset():
        for f, f0 in zip(F, F0):
            f.copy_(f0)
        capi.cpd_als_init(h, F, R)

    # eager reference
    reset()
    for _ in range(K):
        capi.cpd_als_iter_async(h, F, lam, R, fit)
    capi.cpd_als_status(h)
    torch.cuda.synchronize()
    ref = [f.clone() for f in F]
    ref_fit = fit.clone()

    g = torch.cuda.CUDAGraph()
    reset()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        for _ in range(K):
            capi.cpd_als_iter_async(h, F, lam, R, fit)
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        capi.cpd_als_status(h)
        for a, b in zip(F, ref):
            assert torch.equal(a, b), f"replay {rep}: factors differ from eager"
        assert torch.equal(fit, ref_fit), f"replay {rep}: fit differs"
        # unrelated eager work between replays
        _ = (torch.rand(1000, device="cuda") * 2).sum().item()
    h.free()


def test_batched_mttkrp_in_graph_matches_eager():
    print("case graph batch", flush=True)
    R = 16
    rng = np.random.default_rng(4)
    ts = [workloads.random_tensor(tuple(int(x) for x in rng.integers(100, 400, 3)), int(rng.integers(500, 30000)),
                                  seed=300 + i) for i in range(10)]
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R)) for t in ts]
    F = [gu.dev_factors(workloads.random_factors(t.dims, R, seed=i)) for i, t in enumerate(ts)]
    outs = [[torch.zeros((d, R), device="cuda") for d in t.dims] for t in ts]
    b = capi.mttkrp_batch_create(hs, R)
    for n in range(3):   # eager first: uploads the descriptors for these pointers
        capi.mttkrp_batch_run(b, n, F, [o[n] for o in outs])
    torch.cuda.synchronize()
    ref = [[o.clone() for o in os_] for os_ in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for n in range(3):
            capi.mttkrp_batch_run(b, n, F, [o[n] for o in outs])
    for rep in range(3):
        for os_ in outs:
            for o in os_:
                o.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(ts)):
            for n in range(3):
                assert torch.equal(outs[i][n], ref[i][n]), f"replay {rep}: tensor {i} mode {n}"
    b.free()
