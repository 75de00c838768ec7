"""The CP-ALS server on the GPU: jobs of different shapes and ranks arrive
over time and share steps; every job's final factors must be bitwise the
same as when it runs alone, the FIFO one-at-a-time executor must agree, and
every served job's fit trajectory must match the FP64 oracle's CP-ALS from
the same starting factors."""

import numpy as np
import pytest

import oracle
import workloads
from paper_2503_18198_amd.serve import CpdServer, GpuExecutor, ServeJob, initial_factors

pytestmark = pytest.mark.gpu


def jobs(specs, first=0):
    """Job i of the list is built from seeds 500 + first + i and first + i, so
    a job rebuilt alone (first = its position) is the same job."""
    out = []
    for i, (dims, nnz, R, arr) in enumerate(specs, start=first):
        t = workloads.random_tensor(dims, nnz, dist="zipf", s=1.2, seed=500 + i)
        out.append(ServeJob(job_id=i, arrival_s=arr, dims=t.dims, R=R, idx=t.idx, val=t.val, nnz=t.nnz, seed=i,
                            max_iters=8, tol=1e-6))
    return out


# 3, 4 and 5 modes at R = 16, 32 and 64: every (N, R) group the serving mix
# has, with two jobs in most groups so their sweeps are batched.
SPECS = [((300, 250, 200), 20000, 16, 0.0), ((400, 300, 350), 30000, 16, 0.0), ((200, 150, 120, 40), 15000, 32, 0.0),
         ((350, 280, 260), 25000, 16, 0.05), ((250, 200, 150, 30), 12000, 32, 0.1), ((500, 400, 300), 40000, 32, 0.2),
         ((120, 100, 90, 80, 70), 15000, 64, 0.0), ((110, 95, 85, 75, 66), 12000, 64, 0.05),
         ((300, 200, 150), 20000, 64, 0.1), ((90, 80, 70, 60, 50), 10000, 16, 0.15)]


@pytest.mark.parametrize("build_threads", [0, 3])
def test_results_same_alone_and_in_the_mix(build_threads):
    """Also with layout builds on worker threads, overlapping the sweeps of
    jobs already running."""
    print(f"case serve mix, {build_threads} build threads", flush=True)
    mix = jobs(SPECS)
    m = CpdServer(GpuExecutor(batched=True), hbm_budget_bytes=8 << 30, max_slots=16,
                  build_threads=build_threads).run(mix)
    assert m["completed"] == len(SPECS), m
    for i in range(len(SPECS)):
        alone = jobs([SPECS[i]], first=i)[0]
        alone.arrival_s = 0.0
        CpdServer(GpuExecutor(batched=True), hbm_budget_bytes=8 << 30, max_slots=16).run([alone])
        assert alone.iters == mix[i].iters and alone.fits == mix[i].fits, i
        for a, b in zip(alone.result["factors"], mix[i].result["factors"]):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"job {i}: factors differ alone vs mix"


def test_fifo_executor_agrees():
    print("case serve fifo", flush=True)
    a = jobs(SPECS[:3])
    b = jobs(SPECS[:3])
    CpdServer(GpuExecutor(batched=True), 8 << 30, 16).run(a)
    CpdServer(GpuExecutor(batched=False), 8 << 30, 1).run(b)
    for x, y in zip(a, b):
        assert x.fits == y.fits
        for p, q in zip(x.result["factors"], y.result["factors"]):
            assert np.array_equal(p, q)


def test_budget_limits_concurrency():
    print("case serve budget", flush=True)
    js = jobs(SPECS[:4])
    ex = GpuExecutor(batched=True)
    one = max(ex.footprint(j) for j in js)
    srv = CpdServer(ex, hbm_budget_bytes=int(one * 1.5), max_slots=16)
    m = srv.run(js)
    assert m["completed"] == 4 and srv.peak_in_use <= int(one * 1.5)


def test_served_fits_match_oracle():
    """Each served job (run in the mix, batched with the others of its (N, R)
    group) against the FP64 oracle's CP-ALS from the same starting factors for
    the same number of sweeps: every fit of the trajectory within 1e-5
    absolute and its final factors within 1e-3 relative Frobenius."""
    print("case serve vs oracle", flush=True)
    mix = jobs(SPECS)
    m = CpdServer(GpuExecutor(batched=True), hbm_budget_bytes=8 << 30, max_slots=16).run(mix)
    assert m["completed"] == len(SPECS), m
    worst = 0.0
    for j in mix:
        F0 = [f.cpu().numpy() for f in initial_factors(j.dims, j.R, j.seed)]
        st = oracle.cp_als(j.idx, j.val, j.dims, F0, n_iter=j.iters, threads=8)
        gap = float(np.max(np.abs(np.array(j.fits) - np.array(st.fits))))
        worst = max(worst, gap)
        print(f"  job {j.job_id} N={len(j.dims)} R={j.R} sweeps {j.iters}: fit {j.fits[-1]:.6f} "
              f"oracle {st.fits[-1]:.6f} max gap {gap:.1e}", flush=True)
        assert len(j.fits) == len(st.fits) and gap <= 1e-5, f"job {j.job_id}"
        for a, b in zip(j.result["factors"], st.factors):
            e = float(np.linalg.norm(a - b) / np.linalg.norm(b))
            assert e <= 1e-3, f"job {j.job_id}: factor rel err {e:.2e}"
    print(f"  worst fit gap {worst:.1e}", flush=True)
