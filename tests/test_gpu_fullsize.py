"""Parity at the benchmark's full size and launch configuration: the
20M-nonzero 200000 x 150000 x 100000 Zipf(1.2) tensor at R=32 with the
library defaults (the launch bench.py times).  The oracle computes sampled
output rows one by one: the 50 heaviest rows of every mode (the longest
accumulations, spread over many partitions and carries) and 200 random ones,
plus every row cut by a partition boundary.  Bar: relative Frobenius error
<= 1e-5 over the sampled rows, and no sampled row above 1e-5 relative."""

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def launch_geometry(nnz, n_in, R, info, max_parts=8192):
    """Nonzeros per lane group and per workgroup partition, and the partition
    count, as the library plans them (groups of R/4 lanes, runs of a multiple
    of 32 nonzeros, parts_per_cu partitions per compute unit)."""
    groups = info["wg_threads"] // (R // 4)
    target = info["parts_per_cu"] * info["cu_count"]
    per_group = -(-nnz // (target * groups))
    gsz = max(32, -(-per_group // 32) * 32)
    parts = -(-nnz // (gsz * groups))
    if parts > max_parts:
        gsz = -(-(-(-nnz // (max_parts * groups))) // 32) * 32
        parts = -(-nnz // (gsz * groups))
    return gsz, gsz * groups, parts


def test_zipf20m_full_size_sampled_rows():
    print("case full-size zipf1.2-20M", flush=True)
    R = 32
    t = workloads.named_tensor("zipf1.2-20M")
    F = workloads.random_factors(t.dims, R, seed=2)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    dF = gu.dev_factors(F)
    F64 = [f.astype(np.float64) for f in F]
    val64 = t.val.astype(np.float64)
    rng = np.random.default_rng(0)
    for n in range(3):
        print(f"  mode {n}", flush=True)
        out = torch.full((t.dims[n], R), float("nan"), device="cuda")
        capi.mttkrp_run(h, n, dF, out, R)
        torch.cuda.synchronize()
        counts = np.bincount(t.idx[:, n].astype(np.int64), minlength=t.dims[n])
        heavy = np.argsort(counts)[-50:]
        # The copy is sorted by output row, so the row holding sorted position
        # k is np.sort(idx[:, n])[k]: rows cut by partition (carry fix-up) and
        # lane-group (in-workgroup combine) boundaries.
        gsz, wgc, nparts = launch_geometry(t.nnz, len(t.dims) - 1, R, capi.mttkrp_layout_info(h))
        srows = np.sort(t.idx[:, n])
        cut_parts = srows[np.arange(1, nparts, dtype=np.int64) * wgc]
        cut_groups = srows[rng.choice(np.arange(1, t.nnz // gsz, dtype=np.int64) * gsz, 200, replace=False)]
        rows = np.unique(np.concatenate([heavy, rng.integers(0, t.dims[n], 200), cut_parts, cut_groups])).astype(np.uint32)
        ref = oracle.mttkrp_rows(t.idx, val64, t.dims, F64, n, rows)
        got = out.cpu().numpy()[rows.astype(np.int64)]
        assert np.all(np.isfinite(got))
        e = gu.rel_fro(got, ref)
        per_row = np.linalg.norm(got - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
        print(f"  mode {n}: rel fro {e:.2e}, worst row {per_row.max():.2e}", flush=True)
        assert e <= 1e-5 and per_row.max() <= 1e-5, f"mode {n}"
    h.free()
