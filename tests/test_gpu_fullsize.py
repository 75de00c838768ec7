"""Parity at the benchmark's full size and launch configurations: the
20M-nonzero 200000 x 150000 x 100000 Zipf(1.2) tensor at R=32, on the
nonzero-ordered copies in the launch shape the single-layout autotuner picks
(as bench.py does before timing), in the 32 / 256 / 4 shape it picked in the
committed profiles, and in the library defaults, and on the hot-steps copies
with 2 partitions per compute unit.  Every output row of every mode is
compared with the FP64 oracle (16 threads, about a second per mode).
Bar: relative Frobenius error <= 1e-5 per mode, and no row whose own
relative error exceeds 1e-5 (rows of tiny norm are judged against the mode's
largest row norm)."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tensor():
    return workloads.named_tensor("zipf1.2-20M")


@pytest.mark.parametrize("layout", ["hot_steps", "nonzero_order", "shape_32_256_4", "autotuned"])
def test_zipf20m_full_size_every_row(tensor, layout):
    print("case full-size zipf1.2-20M, every row,", layout, flush=True)
    R = 32
    t = tensor
    F = workloads.random_factors(t.dims, R, seed=2)
    opts = {"hot_steps": dict(max_R=R, hot_steps=1, parts_per_cu=2),
            "shape_32_256_4": dict(max_R=R, parts_per_cu=32, part_threads=256, part_gathers=4)}.get(
        layout, dict(max_R=R))
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=opts)
    dF = gu.dev_factors(F)
    if layout == "autotuned":
        outs = [torch.empty((d, R), device="cuda") for d in t.dims]
        best, _ = capi.mttkrp_autotune_shape(h, R, dF, outs, reps=3)
        print(f"  autotuned shape {best}", flush=True)
        del outs
    F64 = [f.astype(np.float64) for f in F]
    val64 = t.val.astype(np.float64)
    for n in range(3):
        print(f"  mode {n}", flush=True)
        out = torch.full((t.dims[n], R), float("nan"), device="cuda")
        capi.mttkrp_run(h, n, dF, out, R)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = oracle.mttkrp(t.idx, val64, t.dims, F64, n, threads=16)
        assert np.all(np.isfinite(got)), f"mode {n}: non-finite output"
        e = gu.rel_fro(got, ref)
        rn = np.linalg.norm(ref, axis=1)
        dn = np.linalg.norm(got - ref, axis=1)
        floor = 1e-3 * rn.max()
        per_row = dn / np.maximum(rn, floor)
        empty = rn == 0
        print(f"  mode {n}: rel fro {e:.2e}, worst row {per_row.max():.2e}, "
              f"rows {t.dims[n]}, empty {int(empty.sum())}", flush=True)
        assert e <= 1e-5, f"mode {n}: rel fro {e}"
        assert per_row.max() <= 1e-5, f"mode {n}: row {int(per_row.argmax())} rel err {per_row.max()}"
        assert np.all(got[empty] == 0.0), f"mode {n}: empty rows not zero"
    h.free()
