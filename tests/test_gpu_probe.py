"""The gather-ceiling probe (a measurement aid): all four variants run on
every mode for fp32 and bf16 factor rows (and on 16-bit coordinates), leave
the caller's memory alone, and reject bad arguments like mttkrp_run."""

import numpy as np
import pytest
import torch

import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_probe_runs_and_writes_nothing_of_the_callers():
    print("case probe", flush=True)
    R = 32
    t = workloads.random_tensor((700, 500, 300, 40), 40_000, dist="zipf", s=1.2, seed=8)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    F = gu.dev_factors(workloads.random_factors(t.dims, R, seed=8))
    Fb = [f.to(torch.bfloat16) for f in F]
    before = [f.clone() for f in F]
    for n in range(4):
        for what in (0, 1, 2, 3):
            capi.mttkrp_gather_probe(h, n, F, R, what)
            capi.mttkrp_gather_probe(h, n, Fb, R, what)
    torch.cuda.synchronize()
    for a, b in zip(F, before):
        assert torch.equal(a, b)
    # the MTTKRP after a probe is unaffected (the probe may touch the carry workspace)
    out = torch.empty((t.dims[1], R), device="cuda")
    capi.mttkrp_run(h, 1, F, out, R)
    ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, [f.cpu().numpy() for f in F], 1)
    assert gu.rel_fro(out.cpu().numpy(), ref) <= 1e-5
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_gather_probe(h, 0, F, R, what=4)
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_gather_probe(h, 4, F, R)
    h.free()


def test_split_variants_refused_beyond_four_modes():
    """Variants 2 and 3 are compiled for 3- and 4-mode tensors; a 5-mode
    tensor gets an error from them and still runs variants 0 and 1."""
    print("case probe 5 modes", flush=True)
    R = 16
    t = workloads.random_tensor((60, 50, 40, 30, 20), 5000, seed=9)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    F = gu.dev_factors(workloads.random_factors(t.dims, R, seed=9))
    for what in (0, 1):
        capi.mttkrp_gather_probe(h, 0, F, R, what)
    for what in (2, 3):
        with pytest.raises(capi.MttkrpError):
            capi.mttkrp_gather_probe(h, 0, F, R, what)
    torch.cuda.synchronize()
    out = torch.empty((t.dims[0], R), device="cuda")
    capi.mttkrp_run(h, 0, F, out, R)
    ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, [f.cpu().numpy() for f in F], 0)
    assert gu.rel_fro(out.cpu().numpy(), ref) <= 1e-5
    h.free()
