"""Mode copies built on the device against the same copies built on the host.

The two builds must produce the same arrays in the same order, so every
mode's MTTKRP output (written over NaN) is bitwise equal, and so are the
factors after a CP-ALS sweep.  |X|^2 is reduced in another order on the
device, so the fit may differ in the last bits only.
"""

import numpy as np
import pytest
import torch

import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def coo(dims, nnz, seed, dist="uniform", dup=0, heavy=None):
    if dist == "zipf":
        t = workloads.random_tensor(dims, nnz, dist="zipf", s=1.2, seed=seed)
        idx, val = t.idx.copy(), t.val.copy()
    else:
        t = workloads.random_tensor(dims, nnz, seed=seed)
        idx, val = t.idx.copy(), t.val.copy()
    if heavy is not None:
        idx[: idx.shape[0] // 3, 0] = heavy
    if dup:
        idx[1 : 2 * dup : 2] = idx[0 : 2 * dup - 1 : 2]
    return idx, val


CASES = {
    "uniform3": ((1000, 800, 600), 100_000, "uniform", 0, None),
    "zipf3_empty_rows": ((30_000, 20_000, 10_000), 300_000, "zipf", 0, None),
    "heavy_row_dups": ((500, 400, 300), 50_000, "uniform", 700, 17),
    "five_modes": ((100, 50, 40, 30, 20), 40_000, "uniform", 0, None),
    "dim_one": ((1, 500, 70), 20_000, "uniform", 0, None),
    "key_exactly_64_bits": ((65_536,) * 4, 20_000, "uniform", 0, None),
    "key_80_bits": ((1 << 20,) * 4, 20_000, "uniform", 0, None),
    "key_72_bits_zipf_5_modes": ((9000, 70_000, 100_000, 120, 100_000), 200_000, "zipf", 300, None),
    "key_exactly_128_bits": ((1 << 16,) * 8, 20_000, "uniform", 0, None),
    "key_over_128_bits_host_path": ((1 << 17,) * 8, 20_000, "uniform", 0, None),
}


@pytest.mark.parametrize("nnz", [1, 31, 33, 1000])
def test_ragged_sizes_match_host_build(nnz):
    print(f"case device layout ragged nnz={nnz}", flush=True)
    idx, val = coo((40, 30, 20), nnz, seed=nnz)
    compare((40, 30, 20), idx, val, R=16)


@pytest.mark.parametrize("case", list(CASES))
def test_device_build_matches_host_build(case):
    dims, nnz, dist, dup, heavy = CASES[case]
    print(f"case device layout {case}", flush=True)
    idx, val = coo(dims, nnz, seed=11, dist=dist, dup=dup, heavy=heavy)
    compare(dims, idx, val, R=32)


def compare(dims, idx, val, R):
    N = len(dims)
    F = workloads.random_factors(dims, R, seed=3)
    hd = capi.mttkrp_layout_build(idx, val, dims, opts=dict(max_R=R))
    hh = capi.mttkrp_layout_build(idx, val, dims, opts=dict(max_R=R, build_on_host=1))
    dF = gu.dev_factors(F)
    for n in range(N):
        a = gu.gpu_mttkrp(hd, n, dF, R)
        b = gu.gpu_mttkrp(hh, n, dF, R)
        assert np.all(np.isfinite(a)), f"mode {n}: unwritten output rows"
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"mode {n}: device and host builds differ"
    # one CP-ALS sweep on each; a degenerate tensor (a single nonzero) makes V
    # singular, and then both builds must report it
    fits, facs, errs = [], [], []
    for h in (hd, hh):
        G = gu.dev_factors(F)
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
        fit = torch.empty(1, dtype=torch.float64, device="cuda")
        capi.cpd_als_init(h, G, R)
        try:
            capi.cpd_als_iter(h, G, lam, R, fit)
            errs.append(None)
        except capi.MttkrpError as ex:
            errs.append(ex.status)
        torch.cuda.synchronize()
        fits.append(float(fit.item()))
        facs.append([g.cpu().numpy() for g in G])
    assert errs[0] == errs[1], errs
    if errs[0] is not None:
        hd.free()
        hh.free()
        return
    for a, b in zip(*facs):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), "factors after a sweep differ"
    assert abs(fits[0] - fits[1]) <= 1e-12 * max(1.0, abs(fits[1])), fits
    hd.free()
    hh.free()
