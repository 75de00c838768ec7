"""Tuned launch shapes of the partition kernel (3-mode tensors, fp32 factors):
every workgroup size (256, 512, 1024 threads) and gathers in flight (2, 4) at
R = 16, 32, 64 against the FP64 oracle, on a tensor with one 16-bit and two
32-bit copies and a ragged nonzero count; bf16 runs ignore the shape; a batch
of tuned layouts is bitwise their single runs; the shape autotuner leaves its
choice set; scheme 2 and scheme 1 partitions with a tuned shape."""

import functools

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

TOL = 1e-5
SHAPES = [(t, u) for t in (256, 512, 1024) for u in (2, 4)]
DIMS = (3000, 2000, 70000)   # copy 2 stores 16-bit coordinates, copies 0 and 1 32-bit


@functools.lru_cache(maxsize=None)
def case(R):
    t = workloads.random_tensor(DIMS, 150_001, dist="zipf", s=1.2, seed=61)
    F = workloads.random_factors(t.dims, R, seed=62)
    refs = [gu.oracle_mttkrp(t.idx, t.val, t.dims, F, n) for n in range(3)]
    return t, F, refs


@pytest.mark.parametrize("R", [16, 32, 64])
@pytest.mark.parametrize("threads,gathers", SHAPES)
def test_shape_matches_oracle(threads, gathers, R):
    print("case shape", threads, gathers, "R", R, flush=True)
    t, F, refs = case(R)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims,
                                 opts=dict(max_R=R, part_threads=threads, part_gathers=gathers, parts_per_cu=4))
    info = capi.mttkrp_layout_info(h)
    assert info["wg_threads"] == threads and info["gathers_in_flight"] == gathers
    assert info["idx16_modes"] == 0b100
    dF = gu.dev_factors(F)
    for n in range(3):
        a = gu.gpu_mttkrp(h, n, dF, R)
        b = gu.gpu_mttkrp(h, n, dF, R)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"mode {n}: runs differ"
        e = gu.rel_fro(a, refs[n])
        assert e <= TOL, f"mode {n}: rel err {e:.3e}"
    h.free()


def test_bf16_runs_ignore_the_shape():
    """The tuned shape applies to fp32 runs only: a bf16 run on a tuned layout
    is bitwise the bf16 run on a default one."""
    print("case shape bf16", flush=True)
    R = 32
    t, F, _ = case(R)
    ht = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, part_threads=1024, part_gathers=2))
    hd = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    dF = gu.dev_factors(F, dtype=torch.bfloat16)
    for n in range(3):
        a = gu.gpu_mttkrp(ht, n, dF, R, bf16=True)
        b = gu.gpu_mttkrp(hd, n, dF, R, bf16=True)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"mode {n}"
    ht.free()
    hd.free()


def tuned_batch(shape, R=32, count=8, seed=70):
    rng = np.random.default_rng(seed)
    ts = []
    for i in range(count):
        dims = tuple(int(x) for x in rng.integers(100, 3000, size=3))
        nnz = 0 if i == 3 else int(np.exp(rng.uniform(np.log(50), np.log(200_000))))
        ts.append(workloads.random_tensor(dims, nnz, dist="zipf", s=1.2, seed=seed + 100 + i))
    ppc, th, gu_ = shape
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims,
                                   opts=dict(max_R=R, parts_per_cu=ppc, part_threads=th, part_gathers=gu_))
          for t in ts]
    F = [workloads.random_factors(t.dims, R, seed=seed + 200 + i) for i, t in enumerate(ts)]
    return ts, hs, F, [gu.dev_factors(f) for f in F]


@pytest.mark.parametrize("shape", [(2, 1024, 2), (4, 256, 4), (1, 512, 2)])
def test_tuned_batch_matches_single_and_oracle(shape):
    print("case shape batch", shape, flush=True)
    R = 32
    ts, hs, F, dF = tuned_batch(shape, R)
    b = capi.mttkrp_batch_create(hs, R)
    for n in range(3):
        outs = [torch.full((t.dims[n], R), float("nan"), device="cuda") for t in ts]
        capi.mttkrp_batch_run(b, n, dF, outs)
        torch.cuda.synchronize()
        for i, t in enumerate(ts):
            got = outs[i].cpu().numpy()
            assert np.array_equal(got.view(np.uint32), gu.gpu_mttkrp(hs[i], n, dF[i], R).view(np.uint32)), \
                f"tensor {i} mode {n}: batched differs from single"
            assert gu.rel_fro(got, gu.oracle_mttkrp(t.idx, t.val, t.dims, F[i], n)) <= TOL
    b.free()
    for h in hs:
        h.free()


def test_batch_refuses_mixed_shapes():
    print("case shape mixed", flush=True)
    t = workloads.random_tensor((300, 200, 100), 5000, seed=5)
    h1 = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=16, part_threads=256))
    h2 = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=16, part_threads=1024))
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_batch_create([h1, h2], 16)
    h1.free()
    h2.free()


def test_shape_autotuner_sets_its_choice():
    print("case shape autotune", flush=True)
    R = 16
    ts, hs, F, dF = tuned_batch((8, 0, 0), R, count=6, seed=90)
    outs = [[torch.empty((d, R), device="cuda") for d in t.dims] for t in ts]
    cands = [(2, 256, 2), (4, 1024, 4), (8, 0, 0), (1, 512, 4)]
    best, times = capi.mttkrp_batch_autotune_shape(hs, R, dF, outs, candidates=cands, reps=2)
    assert best in cands and set(times) == set(cands) and all(v > 0 for v in times.values())
    assert times[best] == min(times.values())
    for h in hs:
        info = capi.mttkrp_layout_info(h)
        assert info["parts_per_cu"] == best[0]
        assert info["wg_threads"] == (best[1] or 512)
    b = capi.mttkrp_batch_create(hs, R)
    for n in range(3):
        o = [torch.full((t.dims[n], R), float("nan"), device="cuda") for t in ts]
        capi.mttkrp_batch_run(b, n, dF, o)
        torch.cuda.synchronize()
        for i, t in enumerate(ts):
            assert gu.rel_fro(o[i].cpu().numpy(), gu.oracle_mttkrp(t.idx, t.val, t.dims, F[i], n)) <= TOL
    b.free()
    defaults = capi.mttkrp_batch_autotune_default_shapes(3)
    assert len(defaults) == 36 and (8, 512, 4) in defaults
    for h in hs:
        h.free()


@pytest.mark.parametrize("opts", [dict(part_threads=1024, part_gathers=4),
                                  dict(part_threads=256, part_gathers=2, partitioner=capi.MTTKRP_PART_ROWS_LPT,
                                       lpt_parts=300)])
def test_scheme2_and_scheme1_with_a_tuned_shape(opts):
    print("case shape schemes", opts, flush=True)
    R = 32
    t, F, refs = case(R)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, **opts))
    dF = gu.dev_factors(F)
    for n in range(3):
        out = torch.full((t.dims[n], R), float("nan"), device="cuda")
        if opts.get("partitioner"):
            capi.mttkrp_run(h, n, dF, out, R)
        else:
            capi.mttkrp_run_scheme2(h, n, dF, out, R)
        torch.cuda.synchronize()
        e = gu.rel_fro(out.cpu().numpy(), refs[n])
        assert e <= TOL, f"mode {n}: rel err {e:.3e}"
    h.free()


def test_cp_als_on_a_tuned_layout_matches_oracle():
    print("case shape cp-als", flush=True)
    R = 16
    t = workloads.random_tensor((400, 300, 200), 30_000, dist="zipf", s=1.2, seed=77)
    F0 = workloads.random_factors(t.dims, R, seed=78)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, part_threads=256, part_gathers=4))
    d = gu.dev_factors(F0)
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")
    capi.cpd_als_init(h, d, R)
    fits = []
    for _ in range(4):
        capi.cpd_als_iter(h, d, lam, R, fit)
        fits.append(float(fit.item()))
    st = oracle.cp_als(t.idx, t.val, t.dims, F0, n_iter=4, threads=8)
    assert max(abs(a - b) for a, b in zip(fits, st.fits)) <= 1e-5
    h.free()


def test_single_layout_shape_autotuner():
    """mttkrp_autotune_shape on one layout: the fastest candidate is set and
    mttkrp_run then matches the oracle and repeats bitwise; refused on
    hot-steps copies."""
    print("case shape autotune single", flush=True)
    R = 32
    t, F, refs = case(R)
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R))
    dF = gu.dev_factors(F)
    outs = [torch.empty((d, R), device="cuda") for d in t.dims]
    cands = [(16, 256, 4), (8, 0, 0), (4, 1024, 2)]
    best, times = capi.mttkrp_autotune_shape(h, R, dF, outs, candidates=cands, reps=2)
    assert best in cands and times[best] == min(times.values())
    info = capi.mttkrp_layout_info(h)
    assert (info["parts_per_cu"], info["wg_threads"]) == (best[0], best[1] or 512)
    for n in range(3):
        a = gu.gpu_mttkrp(h, n, dF, R)
        assert np.array_equal(a.view(np.uint32), gu.gpu_mttkrp(h, n, dF, R).view(np.uint32))
        assert gu.rel_fro(a, refs[n]) <= TOL
    h.free()
    hs = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, hot_steps=1))
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_autotune_shape(hs, R, dF, outs, candidates=cands, reps=1)
    hs.free()


def test_autotuner_second_stage_with_more_than_four_candidates():
    """With more than four candidates the four fastest are timed again; the
    choice is one of the candidates, every time is positive and the layouts
    end on the choice."""
    print("case shape autotune two stages", flush=True)
    R = 32
    ts, hs, F, dF = tuned_batch((8, 0, 0), R, count=5, seed=95)
    outs = [[torch.empty((d, R), device="cuda") for d in t.dims] for t in ts]
    cands = [(1, 256, 2), (2, 512, 4), (4, 1024, 2), (8, 0, 0), (16, 256, 4), (32, 512, 2)]
    best, times = capi.mttkrp_batch_autotune_shape(hs, R, dF, outs, candidates=cands, reps=2)
    assert best in cands and len(times) == 6 and all(v > 0 for v in times.values())
    for h in hs:
        info = capi.mttkrp_layout_info(h)
        assert (info["parts_per_cu"], info["wg_threads"]) == (best[0], best[1] or 512)
    for h in hs:
        h.free()
