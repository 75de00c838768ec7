"""Oracle BF16 rounding against torch's CPU conversion; generator properties."""

import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from workloads import gen


def test_bf16_round_matches_torch_cpu():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(200000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 200000).astype(np.float32),
        rng.uniform(-1, 1, 100000).astype(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 3.3895314e38, -3.3895314e38, 1e-40, -1e-40, 1.0, -1.0],
                 dtype=np.float32),
    ])
    # exact ties: low 16 bits == 0x8000, with both parities of the kept bit
    bits = rng.integers(0, 2 ** 31, 50000, dtype=np.uint64).astype(np.uint32)
    ties = ((bits & np.uint32(0xFFFF0000)) | np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, ties[np.isfinite(ties)]])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = oracle.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_bf16_round_nan_stays_nan():
    x = np.array([np.nan, -np.nan], dtype=np.float32)
    assert np.all(np.isnan(oracle.bf16_round(x)))


def test_bf16_relative_error_bound():
    x = np.random.default_rng(1).uniform(1e-3, 1e3, 100000).astype(np.float32)
    r = oracle.bf16_round(x)
    assert np.max(np.abs(r - x) / x) <= 2.0 ** -8


# ----------------------------------------------------------------- generators
def test_zipf_rank_frequency_slope():
    """Raw Zipf(s) draws: the log-log rank-frequency slope is -s within 0.05."""
    for s in (1.1, 1.2):
        rng = np.random.default_rng(5)
        cdf = gen.zipf_cdf(20000, s)
        r = gen.zipf_ranks(rng, cdf, 4_000_000)
        cnt = np.bincount(r, minlength=20000)[:1000].astype(np.float64)
        k = np.arange(1, 1001, dtype=np.float64)
        slope = np.polyfit(np.log(k), np.log(cnt), 1)[0]
        assert abs(slope + s) <= 0.05, (s, slope)


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_random_tensor_distinct_exact_nnz(dist):
    t = workloads.random_tensor((300, 200, 100), 50000, dist=dist, s=1.2, seed=3)
    assert t.nnz == 50000 and t.idx.dtype == np.uint32 and t.val.dtype == np.float32
    assert np.unique(t.idx, axis=0).shape[0] == 50000
    for m, d in enumerate(t.dims):
        assert t.idx[:, m].max() < d
    t2 = workloads.random_tensor((300, 200, 100), 50000, dist=dist, s=1.2, seed=3)
    assert np.array_equal(t.idx, t2.idx) and np.array_equal(t.val, t2.val)


def test_random_tensor_cap_and_wide_keys():
    t = workloads.random_tensor((4, 5, 6), 1000, seed=1)
    assert t.capped and t.nnz == int(0.1 * 120)
    # product of dims beyond 2**63 uses byte keys; still distinct
    t = workloads.random_tensor((100000,) * 5, 20000, dist="zipf", s=1.2, seed=2)
    assert np.unique(t.idx, axis=0).shape[0] == 20000


def test_lognormal_values_and_factors():
    t = workloads.random_tensor((50, 40, 30, 20), 5000, dist="zipf", s=1.1, values="lognormal", seed=9)
    assert np.all(t.val > 0)
    assert abs(np.median(np.log(t.val.astype(np.float64)))) < 0.1
    F = workloads.random_factors((5, 6), 4, seed=1)
    assert F[0].shape == (5, 4) and F[0].dtype == np.float32 and 0 <= F[1].min() and F[1].max() < 1


def test_batch_and_jobs_shapes():
    ts = workloads.batch_tensors(count=6, nnz_range=(1e3, 1e4))
    assert len(ts) == 6
    for t in ts:
        assert all(100 <= d <= 5000 for d in t.dims)
        assert 0 < t.nnz <= 10000
    jobs = workloads.job_stream(20, rate_per_s=10.0)
    assert all(3 <= len(j.dims) <= 5 for j in jobs)
    assert all(j.R in (16, 32, 64) for j in jobs)
    assert all(jobs[i].arrival_s < jobs[i + 1].arrival_s for i in range(19))
    assert math.isfinite(jobs[-1].arrival_s)


@pytest.mark.parametrize("dims,nnz", [((300, 200, 100), 200_000), ((40, 30, 20, 10), 20_000)])
def test_distinct_coords_bitmap_and_sorted_paths_agree(dims, nnz):
    """Remembering accepted coordinates in a bitmap or in a sorted key array
    gives the same coordinates in the same order, with heavy Zipf collisions
    (many top-up rounds) and with the cap nearly reached."""
    out = []
    for use_bitmap in (True, False):
        r_idx = gen._streams(9)[0]
        samplers = [gen._make_sampler(d, "zipf", 1.2, r_idx) for d in dims]
        out.append(gen.distinct_coords(samplers, dims, nnz, r_idx, use_bitmap=use_bitmap))
    assert np.array_equal(out[0], out[1])
    assert np.unique(out[0], axis=0).shape[0] == nnz
