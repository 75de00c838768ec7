"""Precision: FP32 factors against BF16 factor copies (FP32 products and
accumulation; FP64 Gram matrices and normal-equation solve), both against the
FP64 oracle, on the 4-mode Zipf(1.1) lognormal-valued workload.

Default size: the full 50000 x 40000 x 30000 x 2000, 100M-nonzero workload
(MTTKRP_PRECISION_SCALE=0.1 scales every dimension and nnz by 0.1 for a quick
run).  With MTTKRP_PRECISION_REPORT=<path> the measured errors are written
there as JSON.

Bars, per mode and sampled output row (the heaviest rows and random ones):
FP32 relative Frobenius error <= 1e-5.  BF16: every term val * prod(A_m) is
positive here (lognormal values, U(0,1) factors), so rounding each of the 3
factor values to bfloat16 (relative error <= 2^-8 each) moves every term,
and hence every sum, by a relative amount <= (1 + 2^-8)^3 - 1; plus 1e-5 for
the FP32 accumulation.  CP-ALS: three sweeps from the same start, FP32 and
BF16 fits against the FP64 oracle's fits; FP32 within 1e-4.  BF16 within a
first-order bound: the fit is 1 - |X - Xhat| / |X| and its sensitivity to the
model inner product <X, Xhat> is <X, Xhat> / (|X| |X - Xhat|) per unit of
relative error; rounding the N-1 input factors of every term to bfloat16
moves <X, Xhat> by at most (N-1) 2^-8 relative when the rounding errors all
align, so |fit_bf16 - fit| <= (N-1) 2^-8 <X, Xhat> / (|X| |X - Xhat|),
evaluated on the oracle's final state."""

import json
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_2503_18198_amd import capi
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

SCALE = float(os.environ.get("MTTKRP_PRECISION_SCALE", "1"))
BF16_BOUND = (1 + 2.0 ** -8) ** 3 - 1 + 1e-5


@pytest.fixture(scope="module")
def tensor():
    print(f"case precision workload scale {SCALE}", flush=True)
    return workloads.named_tensor("zipf1.1-100M-4mode", scale=SCALE, progress=lambda m: print(f"  {m}", flush=True))


def sample_rows(t, n, rng):
    counts = np.bincount(t.idx[:, n].astype(np.int64), minlength=t.dims[n])
    heavy = np.argsort(counts)[-40:]
    return np.unique(np.concatenate([heavy, rng.integers(0, t.dims[n], 160)])).astype(np.uint32)


def test_mttkrp_fp32_and_bf16_errors(tensor):
    t = tensor
    N = len(t.dims)
    report = {"scale": SCALE, "nnz": t.nnz, "dims": list(t.dims), "mttkrp": {}}
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=64))
    val64 = t.val.astype(np.float64)
    rng = np.random.default_rng(3)
    for R in (32, 64):
        F = workloads.random_factors(t.dims, R, seed=3)
        F64 = [f.astype(np.float64) for f in F]
        d32 = gu.dev_factors(F)
        d16 = gu.dev_factors(F, dtype=torch.bfloat16)
        rows_err = []
        for n in range(N):
            print(f"  R={R} mode {n}", flush=True)
            rows = sample_rows(t, n, rng)
            ref = oracle.mttkrp_rows(t.idx, val64, t.dims, F64, n, rows)
            got32 = gu.gpu_mttkrp(h, n, d32, R)[rows.astype(np.int64)]
            got16 = gu.gpu_mttkrp(h, n, d16, R, bf16=True)[rows.astype(np.int64)]
            e32 = gu.rel_fro(got32, ref)
            e16 = gu.rel_fro(got16, ref)
            row16 = np.abs(got16 - ref).max(axis=1) / np.abs(ref).max(axis=1)
            elem16 = float(np.max(np.abs(got16 - ref) / np.abs(ref)))
            rows_err.append({"mode": n, "fp32_rel_fro": e32, "bf16_rel_fro": e16, "bf16_max_rel_elem": elem16})
            print(f"    fp32 {e32:.2e}  bf16 {e16:.2e} (max elem {elem16:.2e})", flush=True)
            assert e32 <= 1e-5, f"R={R} mode {n}: fp32 {e32:.3e}"
            assert elem16 <= BF16_BOUND, f"R={R} mode {n}: bf16 element error {elem16:.3e} > {BF16_BOUND:.3e}"
            assert np.all(np.isfinite(row16))
        report["mttkrp"][f"R{R}"] = rows_err
    h.free()
    _write(report, "mttkrp")


def test_als_fits_fp32_bf16_vs_oracle(tensor):
    t = tensor
    R = 32
    iters = 3
    F0 = workloads.random_factors(t.dims, R, seed=5)
    print("  oracle CP-ALS", flush=True)
    st = oracle.cp_als(t.idx, t.val.astype(np.float64), t.dims, [f.astype(np.float64) for f in F0], iters,
                       threads=oracle.ref.default_threads())
    fits = {"oracle_fp64": [float(f) for f in st.fits]}
    for name, dt in (("fp32", capi.MTTKRP_FP32), ("bf16", capi.MTTKRP_BF16)):
        print(f"  GPU CP-ALS {name}", flush=True)
        h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, factor_dtype=dt))
        dF = gu.dev_factors(F0)
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
        fit = torch.empty(1, dtype=torch.float64, device="cuda")
        capi.cpd_als_init(h, dF, R)
        got = []
        for _ in range(iters):
            capi.cpd_als_iter(h, dF, lam, R, fit)
            got.append(float(fit.item()))
        fits[name] = got
        h.free()
    gap32 = max(abs(a - b) for a, b in zip(fits["fp32"], fits["oracle_fp64"]))
    gap16 = max(abs(a - b) for a, b in zip(fits["bf16"], fits["oracle_fp64"]))
    print(f"  fits {json.dumps(fits)}; max |fit - oracle|: fp32 {gap32:.2e}, bf16 {gap16:.2e}", flush=True)
    N = len(t.dims)
    xhat2 = float(st.lam @ oracle.hadamard_of_grams(st.grams) @ st.lam)
    res = (1.0 - st.fits[-1]) * np.sqrt(st.normX2)
    inner = 0.5 * (st.normX2 + xhat2 - res * res)
    bound16 = (N - 1) * 2.0 ** -8 * inner / (np.sqrt(st.normX2) * res)
    print(f"  bf16 fit bound {bound16:.2e} (<X,Xhat>/|X|^2 = {inner / st.normX2:.3f})", flush=True)
    _write({"als_R32": fits, "max_fit_gap": {"fp32": gap32, "bf16": gap16}, "bf16_bound": bound16}, "als")
    assert gap32 <= 1e-4
    assert gap16 <= bound16


def _write(obj, key):
    path = os.environ.get("MTTKRP_PRECISION_REPORT")
    if not path:
        return
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key] = obj
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
