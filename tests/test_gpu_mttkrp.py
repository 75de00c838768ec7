"""GPU parity of the per-mode MTTKRP against the FP64 oracle.

Bar: relative Frobenius error <= 1e-5 per mode for FP32 factors.  BF16
factors: <= 1e-5 against the oracle fed the same bf16-rounded factors, and
within (1 + 2^-8)^(N-1) - 1 (+ accumulation slack) of the FP32-factor oracle
for non-negative data.  Results must repeat bit for bit, and must not depend
on the partition count beyond rounding.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

TOL = 1e-5


def build(t, **opts):
    return capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=opts or None)


def check_all_modes(t, R, seed=0, tol=TOL, **opts):
    F = workloads.random_factors(t.dims, R, seed=seed)
    h = build(t, **opts)
    dF = gu.dev_factors(F)
    errs = []
    for n in range(len(t.dims)):
        got = gu.gpu_mttkrp(h, n, dF, R)
        ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, F, n)
        assert np.all(np.isfinite(got)), f"mode {n}: unwritten or non-finite output"
        e = gu.rel_fro(got, ref)
        errs.append(e)
        assert e <= tol, f"mode {n} R={R}: rel err {e:.3e}"
    h.free()
    return errs


@pytest.mark.parametrize("R", [16, 32, 64])
def test_small_uniform_3mode(R):
    t = workloads.random_tensor((1000, 800, 600), 100_000, seed=1)
    print("case small_uniform_3mode R", R, flush=True)
    check_all_modes(t, R)


@pytest.mark.parametrize("dims", [(60, 50, 40, 30), (30, 25, 20, 15, 12), (12, 11, 10, 9, 8, 7, 6, 5)])
def test_more_modes(dims):
    print("case more_modes", dims, flush=True)
    t = workloads.random_tensor(dims, 20_000, dist="zipf", s=1.1, seed=2)
    check_all_modes(t, 32)


def test_zipf_skew_heavy_rows():
    """Zipf(1.2): some rows hold a large share of the nonzeros and span many
    partitions (carry fix-up over many workgroups)."""
    print("case zipf_skew_heavy_rows", flush=True)
    t = workloads.random_tensor((20_000, 15_000, 10_000), 1_000_000, dist="zipf", s=1.2, seed=3)
    for R in (16, 32):
        check_all_modes(t, R)


def test_single_row_holds_everything():
    rng = np.random.default_rng(4)
    nnz = 300_000
    dims = (50, 3000, 2000)
    idx = np.stack([np.full(nnz, 7), rng.integers(0, 3000, nnz), rng.integers(0, 2000, nnz)], axis=1).astype(np.uint32)
    t = workloads.SparseTensor(idx=idx, val=rng.random(nnz).astype(np.float32), dims=dims, nnz_requested=nnz)
    print("case single_row", flush=True)
    for ppc in (1, 8, 64):
        check_all_modes(t, 32, parts_per_cu=ppc)


@pytest.mark.parametrize("R,threads", [(16, 256), (32, 512), (64, 256)])
def test_rows_spanning_hundreds_of_partitions(R, threads):
    """Cut rows longer than the fix-up's 64-partition chunks: a row with 40 %
    of the nonzeros first, ending exactly on a partition boundary, another
    with 25 % in the middle, and many short rows, at 32 and 64 partitions
    per CU (up to a few thousand partitions)."""
    print("case long cut rows", R, threads, flush=True)
    rng = np.random.default_rng(40 + R)
    nnz = 2_000_000
    dims = (3000, 2500, 1800)
    # Row 5 ends at 391 * 2048, a multiple of every partition size used here.
    rows = np.concatenate([np.full(800_768, 5), rng.integers(6, 1500, 399_232), np.full(500_000, 1500),
                           rng.integers(1501, 3000, 300_000)])
    rows.sort()
    idx = np.stack([rows, rng.integers(0, dims[1], nnz), rng.integers(0, dims[2], nnz)], axis=1).astype(np.uint32)
    t = workloads.SparseTensor(idx=idx, val=rng.random(nnz).astype(np.float32), dims=dims, nnz_requested=nnz)
    F = workloads.random_factors(t.dims, R, seed=3)
    dF = gu.dev_factors(F)
    ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, F, 0)
    for ppc in (32, 64):
        h = capi.mttkrp_layout_build(t.idx, t.val, t.dims,
                                     opts=dict(max_R=R, parts_per_cu=ppc, part_threads=threads, build_on_host=1))
        a = gu.gpu_mttkrp(h, 0, dF, R)
        b = gu.gpu_mttkrp(h, 0, dF, R)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"ppc {ppc}: not repeatable"
        e = gu.rel_fro(a, ref)
        rn = np.linalg.norm(ref, axis=1)
        per_row = np.linalg.norm(a - ref, axis=1) / np.maximum(rn, 1e-30)
        assert e <= TOL and per_row[rn > 0].max() <= TOL, f"ppc {ppc}: rel err {e:.3e}, worst row {per_row.max():.3e}"
        h.free()


@pytest.mark.parametrize("nnz", [0, 1, 5, 31, 32, 33, 1000])
def test_tiny_and_ragged(nnz):
    print("case tiny_and_ragged", nnz, flush=True)
    rng = np.random.default_rng(5 + nnz)
    dims = (40, 1, 37)
    idx = np.stack([rng.integers(0, d, nnz) for d in dims], axis=1).astype(np.uint32).reshape(nnz, 3)
    t = workloads.SparseTensor(idx=idx, val=rng.standard_normal(nnz).astype(np.float32), dims=dims,
                               nnz_requested=nnz)
    check_all_modes(t, 16)


def test_duplicates_add_up():
    print("case duplicates", flush=True)
    rng = np.random.default_rng(6)
    dims = (200, 150, 100)
    base = np.stack([rng.integers(0, d, 5000) for d in dims], axis=1).astype(np.uint32)
    idx = np.concatenate([base, base[:2000], base[:100]], axis=0)
    t = workloads.SparseTensor(idx=idx, val=rng.standard_normal(idx.shape[0]).astype(np.float32), dims=dims,
                               nnz_requested=idx.shape[0])
    check_all_modes(t, 32)


def test_deterministic_and_partition_invariant():
    print("case determinism", flush=True)
    t = workloads.random_tensor((5000, 4000, 3000), 400_000, dist="zipf", s=1.2, seed=7)
    R = 32
    F = workloads.random_factors(t.dims, R, seed=1)
    dF = gu.dev_factors(F)
    outs = {}
    for ppc in (1, 8, 64):
        h = build(t, parts_per_cu=ppc)
        a = [gu.gpu_mttkrp(h, n, dF, R) for n in range(3)]
        b = [gu.gpu_mttkrp(h, n, dF, R) for n in range(3)]
        for n in range(3):
            assert np.array_equal(a[n].view(np.uint32), b[n].view(np.uint32)), f"mode {n} not repeatable"
        outs[ppc] = a
        h.free()
    for n in range(3):
        ref = gu.oracle_mttkrp(t.idx, t.val, t.dims, F, n)
        for ppc in outs:
            assert gu.rel_fro(outs[ppc][n], ref) <= TOL


@pytest.mark.parametrize("R", [16, 32, 64])
def test_bf16_factors(R):
    print("case bf16 R", R, flush=True)
    t = workloads.random_tensor((3000, 2500, 2000), 300_000, dist="zipf", s=1.2, seed=8)
    F = workloads.random_factors(t.dims, R, seed=2)
    h = build(t)
    dF = gu.dev_factors(F, dtype=torch.bfloat16)
    Fr = [oracle.bf16_round(f) for f in F]
    bound = (1 + 2.0 ** -8) ** 2 - 1 + 1e-5
    for n in range(3):
        got = gu.gpu_mttkrp(h, n, dF, R, bf16=True)
        exact = gu.oracle_mttkrp(t.idx, t.val, t.dims, Fr, n)
        e = gu.rel_fro(got, exact)
        assert e <= TOL, f"bf16 exact-input parity mode {n}: {e:.3e}"
        full = gu.oracle_mttkrp(t.idx, t.val, t.dims, F, n)
        rel = np.abs(got - full) / np.maximum(np.abs(full), 1e-30)
        assert np.max(rel[full > 0]) <= bound, f"bf16 bound mode {n}: {np.max(rel):.3e} > {bound:.3e}"
        print(f"bf16 R={R} mode {n}: exact-input err {e:.2e}, vs fp32 factors max rel {np.max(rel):.2e}")
    h.free()


def test_argument_errors_on_device():
    t = workloads.random_tensor((100, 90, 80), 1000, seed=9)
    h = build(t)
    F = gu.dev_factors(workloads.random_factors(t.dims, 32, seed=3))
    out = torch.zeros((100, 32), device="cuda")
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_run(h, 3, F, out, 32)
    assert e.value.status == capi.MTTKRP_EINVAL
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_run(h, 0, F, torch.zeros((100, 48), device="cuda"), 48)
    small = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=16))
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_run(small, 0, F, out, 32)
    assert e.value.status == capi.MTTKRP_EINVAL
    # misaligned factor pointer
    bad = torch.zeros(90 * 32 + 1, device="cuda")[1:].view(90, 32)
    with pytest.raises(capi.MttkrpError):
        capi._check(capi._lib.mttkrp_run(__import__("ctypes").c_void_p(h.ptr), 0,
                                         capi._ptr_array([None, bad, F[2]], 3),
                                         __import__("ctypes").c_void_p(out.data_ptr()), 32,
                                         __import__("ctypes").c_void_p(0)))
    h.free()
    small.free()


def test_scheme2_atomics_agrees():
    """The paper's scheme 2 (global atomics for rows cut by partitions), kept
    for comparison, matches the oracle on a skewed tensor with many cut rows
    and on modes with fewer indices than partitions."""
    print("case scheme2", flush=True)
    t = workloads.random_tensor((300, 24, 77, 17), 200_000, dist="zipf", s=1.2, seed=12)
    R = 32
    F = workloads.random_factors(t.dims, R, seed=12)
    dF = gu.dev_factors(F)
    h = build(t, parts_per_cu=8)
    for n in range(4):
        out = torch.full((t.dims[n], R), float("nan"), device="cuda")
        capi.mttkrp_run_scheme2(h, n, dF, out, R)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got)), f"mode {n}: unwritten output"
        e = gu.rel_fro(got, gu.oracle_mttkrp(t.idx, t.val, t.dims, F, n))
        assert e <= TOL, f"mode {n}: {e:.3e}"
    h.free()


@pytest.mark.parametrize("dims,R", [((30, 25, 20, 15, 12), 64), ((12, 11, 10, 9, 8, 7, 6, 5), 32),
                                    ((12, 11, 10, 9, 8, 7, 6, 5), 64)])
def test_bf16_many_modes(dims, R):
    """bf16 rows with 8 values per lane on the widest per-nonzero state (up to
    7 input factors), against the oracle fed the same bf16-rounded factors."""
    print("case bf16 many modes", dims, R, flush=True)
    t = workloads.random_tensor(dims, 30_000, dist="zipf", s=1.1, seed=9)
    F = workloads.random_factors(t.dims, R, seed=9)
    Fr = [oracle.bf16_round(f) for f in F]
    h = build(t)
    dF = gu.dev_factors(F, dtype=torch.bfloat16)
    for n in range(len(dims)):
        got = gu.gpu_mttkrp(h, n, dF, R, bf16=True)
        e = gu.rel_fro(got, gu.oracle_mttkrp(t.idx, t.val, t.dims, Fr, n))
        assert e <= TOL, f"bf16 mode {n}: {e:.3e}"
    h.free()


@pytest.mark.parametrize("dims,R,bf16", [((3000, 2500, 2000), 16, False), ((3000, 2500, 2000), 32, False),
                                         ((3000, 2500, 2000), 64, False), ((3000, 2500, 2000), 32, True),
                                         ((3000, 2500, 2000), 64, True), ((800, 700, 600, 500), 32, False),
                                         ((800, 700, 600, 500), 32, True)])
def test_hot_row_cache(dims, R, bf16):
    """The optional LDS hot-row cache: the most gathered rows of every input
    factor come from LDS, the rest from global memory, in the same launch."""
    print("case hot rows", dims, R, bf16, flush=True)
    t = workloads.random_tensor(dims, 300_000, dist="zipf", s=1.2, seed=13)
    F = workloads.random_factors(t.dims, R, seed=13)
    h = build(t, max_R=R, hot_rows=-1)
    assert capi.mttkrp_layout_info(h)["hot_rows"] > 0
    dF = gu.dev_factors(F, dtype=torch.bfloat16 if bf16 else torch.float32)
    Fr = [oracle.bf16_round(f) for f in F] if bf16 else F
    for n in range(len(dims)):
        got = gu.gpu_mttkrp(h, n, dF, R, bf16=bf16)
        e = gu.rel_fro(got, gu.oracle_mttkrp(t.idx, t.val, t.dims, Fr, n))
        assert e <= TOL, f"mode {n}: {e:.3e}"
    h.free()
