"""Scheduling logic of the CP-ALS server on the CPU, with a fake executor and
a virtual clock: admission by memory and slots in arrival order, retirement
on convergence or iteration cap, memory accounting, and latency statistics."""

import math

import numpy as np
import pytest

from paper_2503_18198_amd.serve import CpdServer, Executor, ServeJob, percentile


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor(Executor):
    """Each step costs `dt` of virtual time; job j's fit after k sweeps is
    1 - rate_j ** k, so it converges after a known number of sweeps."""

    def __init__(self, clock, dt=0.01, budget_check=None):
        self.clock = clock
        self.dt = dt
        self.live = {}
        self.budget_check = budget_check
        self.max_live = 0

    def footprint(self, job):
        return job.nnz * 10

    def admit(self, job):
        self.live[job.job_id] = 0
        self.max_live = max(self.max_live, len(self.live))
        if self.budget_check:
            self.budget_check()
        return job

    def step(self, slots):
        self.clock.t += self.dt
        out = []
        for job in slots:
            self.live[job.job_id] += 1
            rate = 0.3 + 0.05 * (job.job_id % 5)
            out.append(1.0 - rate ** self.live[job.job_id])
        return out

    def release(self, job):
        k = self.live.pop(job.job_id)
        return {"sweeps": k}


def make_jobs(n, gap=0.005, nnz=100):
    return [ServeJob(job_id=i, arrival_s=i * gap, dims=(10, 10, 10), R=16, nnz=nnz + 10 * i, tol=1e-4,
                     max_iters=50) for i in range(n)]


def test_all_jobs_complete_and_converge():
    c = Clock()
    ex = FakeExecutor(c)
    srv = CpdServer(ex, hbm_budget_bytes=10 ** 9, max_slots=8, clock=c, sleep=c.sleep)
    jobs = make_jobs(20)
    m = srv.run(jobs)
    assert m["completed"] == 20 and m["rejected"] == 0
    for j in jobs:
        rate = 0.3 + 0.05 * (j.job_id % 5)
        # converged when the fit change rate^(k-1) (1 - rate) drops below tol
        k = next(k for k in range(2, 60) if rate ** (k - 1) * (1 - rate) < 1e-4)
        assert j.status == "converged" and j.iters == k, (j.job_id, j.iters, k)
        assert j.admitted_s >= j.arrival_s and j.finished_s > j.admitted_s
    assert ex.max_live <= 8


def test_memory_budget_is_never_exceeded():
    c = Clock()
    srv = None

    def check():
        assert srv.in_use <= srv.budget

    ex = FakeExecutor(c, budget_check=check)
    srv = CpdServer(ex, hbm_budget_bytes=5000, max_slots=100, clock=c, sleep=c.sleep)
    jobs = make_jobs(30, gap=0.0, nnz=100)      # footprints 1000..3900 bytes
    m = srv.run(jobs)
    assert m["completed"] == 30
    assert srv.peak_in_use <= 5000
    assert srv.in_use == 0
    # admission follows arrival order
    admits = [jid for _, ev, jid in srv.log if ev == "admit"]
    assert admits == sorted(admits)


def test_oversized_job_is_rejected_not_stuck():
    c = Clock()
    ex = FakeExecutor(c)
    srv = CpdServer(ex, hbm_budget_bytes=2000, max_slots=4, clock=c, sleep=c.sleep)
    jobs = make_jobs(3, nnz=100)
    jobs[1].nnz = 10 ** 6
    m = srv.run(jobs)
    assert m["rejected"] == 1 and m["completed"] == 2
    assert jobs[1].status.startswith("rejected")


def test_iteration_cap_and_failure():
    c = Clock()

    class Stubborn(FakeExecutor):
        def step(self, slots):
            self.clock.t += self.dt
            return [0.5 + 0.01 * len(slots[0].fits) if j.job_id == 0 else float("nan") for j in slots]

    ex = Stubborn(c)
    jobs = make_jobs(2)
    jobs[0].max_iters = 7
    m = CpdServer(ex, 10 ** 9, 4, clock=c, sleep=c.sleep).run(jobs)
    assert jobs[0].status == "max_iters" and jobs[0].iters == 7
    assert jobs[1].status.startswith("failed")
    assert m["completed"] == 1 and m["failed"] == 1


def test_late_arrivals_join_running_steps():
    """A job arriving while others run is admitted at the next step (continuous
    batching), not after the running ones finish."""
    c = Clock()
    ex = FakeExecutor(c, dt=0.01)
    jobs = [ServeJob(0, 0.0, (5, 5, 5), 16, nnz=10, tol=1e-12, max_iters=40),
            ServeJob(1, 0.05, (5, 5, 5), 16, nnz=10, tol=1e-12, max_iters=5)]
    CpdServer(ex, 10 ** 9, 4, clock=c, sleep=c.sleep).run(jobs)
    assert jobs[1].admitted_s < jobs[0].finished_s
    assert jobs[1].finished_s < jobs[0].finished_s


def test_percentiles():
    v = list(range(1, 101))
    assert percentile(v, 50) == pytest.approx(50.5)
    assert percentile(v, 99) == pytest.approx(99.01)
    assert math.isnan(percentile([], 50))
    rng = np.random.default_rng(0)
    x = rng.exponential(size=1001)
    assert percentile(x, 99) == pytest.approx(float(np.sort(x)[990]))
