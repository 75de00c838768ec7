"""Scheduling logic of the CP-ALS server on the CPU, with a fake executor and
a virtual clock: admission by memory and slots in arrival order, retirement
on convergence or iteration cap, memory accounting, and latency statistics."""

import math
import threading
import time

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


class AsyncFakeExecutor(FakeExecutor):
    """Jobs are grouped by rank; a group's sweep takes `dts[R]` of virtual
    time from its launch, and sweeps of different groups overlap."""

    def __init__(self, clock, dts):
        super().__init__(clock)
        self.dts = dts
        self.launches = []          # (time, group, job ids)

    def group_key(self, job):
        return job.R

    def launch(self, key, slots):
        self.launches.append((self.clock.t, key, [j.job_id for j in slots]))
        out = []
        for job in slots:
            self.live[job.job_id] += 1
            rate = 0.3 + 0.05 * (job.job_id % 5)
            out.append(1.0 - rate ** self.live[job.job_id])
        return (self.clock.t + self.dts[key], out)

    def poll(self, token):
        end, out = token
        return out if self.clock.t >= end - 1e-12 else None

    def wait(self, tokens, timeout_s):
        first = min(end for end, _ in tokens)
        self.clock.t = max(self.clock.t, first if timeout_s is None else min(first, self.clock.t + timeout_s))


def test_groups_step_independently():
    """A fast group keeps sweeping while a slow group's sweep runs, so its jobs
    finish in their own sweep count x their own sweep time; every job still
    gets the same fits and iteration count as in lockstep."""
    c = Clock()
    ex = AsyncFakeExecutor(c, {16: 0.001, 64: 0.02})
    jobs = [ServeJob(i, 0.0, (5, 5, 5), 16 if i % 2 else 64, nnz=10, tol=1e-4, max_iters=50) for i in range(6)]
    srv = CpdServer(ex, 10 ** 9, 8, clock=c, sleep=c.sleep)
    m = srv.run(jobs)
    assert m["completed"] == 6
    for j in jobs:
        rate = 0.3 + 0.05 * (j.job_id % 5)
        k = next(k for k in range(2, 60) if rate ** (k - 1) * (1 - rate) < 1e-4)
        assert j.status == "converged" and j.iters == k
        assert j.fits == pytest.approx([1.0 - rate ** i for i in range(1, k + 1)])
        # each job's latency is its own group's sweeps back to back
        assert j.finished_s == pytest.approx(k * ex.dts[j.R], abs=1e-9)
    # at most one sweep per group in flight, and the groups overlap
    for key in (16, 64):
        t = [tt for tt, g, _ in ex.launches if g == key]
        assert all(b - a >= ex.dts[key] - 1e-12 for a, b in zip(t, t[1:]))
    slow_first_end = ex.dts[64]
    assert sum(1 for tt, g, _ in ex.launches if g == 16 and tt < slow_first_end) >= 10


def test_arrival_joins_busy_group_at_its_next_sweep():
    c = Clock()
    ex = AsyncFakeExecutor(c, {16: 0.01})
    jobs = [ServeJob(0, 0.0, (5, 5, 5), 16, nnz=10, tol=1e-12, max_iters=10),
            ServeJob(1, 0.015, (5, 5, 5), 16, nnz=10, tol=1e-12, max_iters=3)]
    CpdServer(ex, 10 ** 9, 4, clock=c, sleep=c.sleep).run(jobs)
    # job 1 is admitted mid-sweep and swept with job 0 from the sweep at t=0.02 on
    assert jobs[1].admitted_s == pytest.approx(0.015)
    assert [ids for tt, _, ids in ex.launches][:4] == [[0], [0], [0, 1], [0, 1]]
    assert jobs[1].finished_s == pytest.approx(0.05) and jobs[0].finished_s == pytest.approx(0.1)


class SlowBuildExecutor(FakeExecutor):
    """Real-time executor: admit (the layout build) sleeps `build_s`, a step
    sleeps `dt`; counts how many admits run at once."""

    def __init__(self, build_s, dt, fail_id=None):
        super().__init__(None, dt=dt)
        self.build_s = build_s
        self.fail_id = fail_id
        self.running = 0
        self.peak_running = 0
        self.lock = threading.Lock()

    def admit(self, job):
        with self.lock:
            self.running += 1
            self.peak_running = max(self.peak_running, self.running)
        time.sleep(self.build_s)
        with self.lock:
            self.running -= 1
        if job.job_id == self.fail_id:
            raise RuntimeError("build failed")
        return super().admit(job)

    def step(self, slots):
        time.sleep(self.dt)
        out = []
        for job in slots:
            self.live[job.job_id] += 1
            rate = 0.3 + 0.05 * (job.job_id % 5)
            out.append(1.0 - rate ** self.live[job.job_id])
        return out


def test_builds_on_worker_threads_overlap_and_give_the_same_results():
    runs = {}
    for threads in (0, 4):
        ex = SlowBuildExecutor(build_s=0.02, dt=0.0005)
        jobs = make_jobs(8, gap=0.0)
        srv = CpdServer(ex, 10 ** 9, 8, build_threads=threads)
        m = srv.run(jobs)
        assert m["completed"] == 8 and srv.in_use == 0
        assert m["admit_s_total"] >= 8 * 0.02 * 0.9
        runs[threads] = (ex.peak_running, [(j.iters, j.fits) for j in jobs])
    assert runs[0][0] == 1 and runs[4][0] >= 2
    assert runs[0][1] == runs[4][1]


@pytest.mark.parametrize("threads", [0, 2])
def test_a_failed_build_fails_that_job_only(threads):
    """A build that raises (say, out of device memory near the budget) marks
    its job failed and hands back its reservation; the other jobs run on."""
    ex = SlowBuildExecutor(build_s=0.001, dt=0.0005, fail_id=2)
    srv = CpdServer(ex, 10 ** 9, 8, build_threads=threads)
    jobs = make_jobs(4, gap=0.0)
    m = srv.run(jobs)
    assert m["failed"] == 1 and m["completed"] == 3
    assert jobs[2].status.startswith("failed: build") and "build failed" in jobs[2].status
    assert all(j.status in ("converged", "max_iters") for j in jobs if j.job_id != 2)
    assert srv.in_use == 0


class ScratchExecutor(SlowBuildExecutor):
    """Each build holds `scratch` transient bytes beside the job's footprint;
    records the server's reservation while builds run."""

    def __init__(self, scratch, **kw):
        super().__init__(**kw)
        self.scratch = scratch
        self.seen = []

    def build_bytes(self, job):
        return self.scratch

    def admit(self, job):
        self.seen.append(self.srv.in_use)
        return super().admit(job)


def test_build_scratch_is_reserved_while_building():
    """Admission counts a job's footprint plus its build scratch; the scratch
    is handed back once the build ends, so afterwards only footprints stay
    reserved, and a budget that fits two builds at once never holds three."""
    fp = 100 * 10 + 10 * 10     # largest footprint of make_jobs(6): nnz * 10
    ex = ScratchExecutor(scratch=5000, build_s=0.01, dt=0.0005)
    budget = 2 * (fp + 5000) + fp // 2
    srv = CpdServer(ex, budget, 8, build_threads=4)
    ex.srv = srv
    jobs = make_jobs(6, gap=0.0)
    m = srv.run(jobs)
    assert m["completed"] == 6 and srv.in_use == 0
    assert ex.peak_running <= 2
    assert srv.peak_in_use <= budget
    assert max(ex.seen) >= 5000   # some build ran while another build's scratch was reserved
