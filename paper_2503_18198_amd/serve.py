"""Continuous-batching CP-ALS server.

Jobs (a sparse tensor, a rank, a stopping rule) arrive over time.  The loop

* admits waiting jobs in arrival order while a slot is free and their device
  footprint (the N mode copies, workspace, factors; ``mttkrp_footprint``)
  fits in what is left of the HBM budget; state then stays on the device;
* runs one scheduler step at a time: one CP-ALS sweep for every active job,
  jobs with the same (N, R) grouped into one batch so their per-mode MTTKRPs
  share one launch pair (``cpd_als_batch_iter_async``);
* after each step reads every active job's fit, retires jobs whose fit
  changed by less than ``tol`` or that reached ``max_iters``, releases their
  memory and admits waiting jobs into the freed room.

Requests that arrive while others run are admitted at the next step, so new
and old jobs share the GPU.  A tensor's results do not depend on which other
jobs share its steps: the batched sweep is bitwise the single-tensor sweep.

The executor is an interface so the scheduling logic can be tested on the
CPU with a fake one.  Latency = completion time - arrival time.
"""

from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class ServeJob:
    job_id: int
    arrival_s: float
    dims: Tuple[int, ...]
    R: int
    idx: Optional[np.ndarray] = None     # (nnz, N) uint32
    val: Optional[np.ndarray] = None     # (nnz,) float32
    nnz: int = 0
    seed: int = 0
    max_iters: int = 50
    tol: float = 1e-4
    # filled by the server
    admitted_s: float = math.nan
    finished_s: float = math.nan
    iters: int = 0
    fits: List[float] = dataclasses.field(default_factory=list)
    result: object = None
    status: str = "pending"

    @property
    def latency_s(self) -> float:
        return self.finished_s - self.arrival_s


class Executor:
    """What the server needs from the device side."""

    def footprint(self, job: ServeJob) -> int:
        raise NotImplementedError

    def admit(self, job: ServeJob):
        """Build the job's device state; returns an opaque slot."""
        raise NotImplementedError

    def step(self, slots: Sequence) -> List[float]:
        """One CP-ALS sweep for every slot; returns their fits (in order)."""
        raise NotImplementedError

    def release(self, slot):
        """Free the slot's device memory; returns the job's result."""
        raise NotImplementedError


def percentile(values: Sequence[float], q: float) -> float:
    """Linear-interpolation percentile (numpy's default definition)."""
    if not len(values):
        return math.nan
    return float(np.percentile(np.asarray(values, dtype=np.float64), q))


class CpdServer:
    def __init__(self, executor: Executor, hbm_budget_bytes: int, max_slots: int = 64,
                 clock: Optional[Callable[[], float]] = None, sleep: Optional[Callable[[float], None]] = None):
        self.ex = executor
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.clock = clock or time.monotonic
        self.sleep = sleep or time.sleep
        self.in_use = 0
        self.peak_in_use = 0
        self.steps = 0
        self.log: List[Tuple[float, str, int]] = []

    def run(self, jobs: Sequence[ServeJob]) -> Dict[str, object]:
        pending = sorted(jobs, key=lambda j: (j.arrival_s, j.job_id))
        waiting: List[ServeJob] = []
        active: List[Tuple[ServeJob, object]] = []
        done: List[ServeJob] = []
        t0 = self.clock()
        pi = 0
        while pi < len(pending) or waiting or active:
            now = self.clock() - t0
            while pi < len(pending) and pending[pi].arrival_s <= now:
                waiting.append(pending[pi])
                pi += 1
            # admission in arrival order, by slot and by memory
            while waiting and len(active) < self.max_slots:
                job = waiting[0]
                need = self.ex.footprint(job)
                if need > self.budget:
                    waiting.pop(0)
                    job.status = "rejected: footprint over the whole budget"
                    job.finished_s = self.clock() - t0
                    done.append(job)
                    self.log.append((job.finished_s, "reject", job.job_id))
                    continue
                if self.in_use + need > self.budget:
                    break
                waiting.pop(0)
                slot = self.ex.admit(job)
                job.admitted_s = self.clock() - t0
                job.status = "running"
                self.in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                active.append((job, slot))
                self.log.append((job.admitted_s, "admit", job.job_id))
            if not active:
                if pi < len(pending):
                    self.sleep(max(0.0, pending[pi].arrival_s - (self.clock() - t0)))
                continue
            fits = self.ex.step([s for _, s in active])
            self.steps += 1
            still = []
            for (job, slot), f in zip(active, fits):
                prev = job.fits[-1] if job.fits else None
                job.fits.append(float(f))
                job.iters += 1
                converged = prev is not None and abs(f - prev) < job.tol
                if not math.isfinite(f):
                    job.status = "failed: non-finite fit"
                elif converged:
                    job.status = "converged"
                elif job.iters >= job.max_iters:
                    job.status = "max_iters"
                if job.status != "running":
                    job.result = self.ex.release(slot)
                    self.in_use -= self.ex.footprint(job)
                    job.finished_s = self.clock() - t0
                    done.append(job)
                    self.log.append((job.finished_s, "retire", job.job_id))
                else:
                    still.append((job, slot))
            active = still
        return self.metrics(done, self.clock() - t0)

    def metrics(self, done: Sequence[ServeJob], makespan: float) -> Dict[str, object]:
        ok = [j for j in done if not j.status.startswith(("rejected", "failed"))]
        lat = [j.latency_s for j in ok]
        return {
            "jobs": len(done),
            "completed": len(ok),
            "rejected": sum(j.status.startswith("rejected") for j in done),
            "failed": sum(j.status.startswith("failed") for j in done),
            "makespan_s": makespan,
            "jobs_per_s": len(ok) / makespan if makespan > 0 else math.nan,
            "p50_latency_s": percentile(lat, 50),
            "p99_latency_s": percentile(lat, 99),
            "mean_latency_s": float(np.mean(lat)) if lat else math.nan,
            "steps": self.steps,
            "peak_hbm_bytes": self.peak_in_use,
        }


class GpuExecutor(Executor):
    """Device state per job: layout handle, fp32 factors, lambda and fit on
    the GPU.  Each step groups the active jobs by (N, R) and runs one batched
    CP-ALS sweep per group of two or more (a lone job runs its own sweep, with
    no batch tables to rebuild); groups use their own streams.  A job's
    results are bitwise the same either way."""

    def __init__(self, batched: bool = True):
        import torch

        from . import capi
        self.torch = torch
        self.capi = capi
        self.batched = batched
        self._batches: Dict[Tuple[int, int], Tuple[tuple, object]] = {}   # group -> (member ids, batch)
        self._streams: Dict[Tuple[int, int], object] = {}
        # Fits of a step are gathered on the device and copied to pinned host
        # memory with one asynchronous copy (a pageable .cpu() costs ~1 ms).
        self._fit_dev = torch.empty(0, dtype=torch.float64, device="cuda")
        self._fit_host = torch.empty(0, dtype=torch.float64)
        self._fit_event = torch.cuda.Event()

    def footprint(self, job: ServeJob) -> int:
        lib = self.capi.mttkrp_footprint(job.dims, job.nnz, opts=dict(max_R=job.R))
        return lib + sum(int(d) * job.R * 4 for d in job.dims) + 16 * job.R

    def admit(self, job: ServeJob):
        torch = self.torch
        h = self.capi.mttkrp_layout_build(job.idx, job.val, job.dims, opts=dict(max_R=job.R))
        rng = np.random.default_rng(job.seed)
        F = [torch.from_numpy(rng.random((d, job.R)).astype(np.float32)).cuda() for d in job.dims]
        lam = torch.zeros(job.R, dtype=torch.float64, device="cuda")
        fit = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.capi.cpd_als_init(h, F, job.R)
        return {"job": job, "h": h, "F": F, "lam": lam, "fit": fit, "key": (len(job.dims), job.R)}

    def _stream(self, key):
        if key not in self._streams:
            self._streams[key] = self.torch.cuda.Stream()
        return self._streams[key]

    def step(self, slots):
        torch = self.torch
        groups: Dict[Tuple[int, int], list] = {}
        for s in slots:
            groups.setdefault(s["key"], []).append(s)
        cur = torch.cuda.current_stream()
        for key, members in groups.items():
            st = self._stream(key)
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                if self.batched and len(members) > 1:
                    ids = tuple(id(m["h"]) for m in members)
                    old = self._batches.get(key)
                    if old is None or old[0] != ids:
                        if old is not None:
                            st.synchronize()
                            old[1].free()
                        self._batches[key] = (ids, self.capi.mttkrp_batch_create([m["h"] for m in members], key[1]))
                    b = self._batches[key][1]
                    self.capi.cpd_als_batch_iter_async(b, [m["F"] for m in members], [m["lam"] for m in members],
                                                       [m["fit"] for m in members], stream=st)
                else:
                    # one job (or no batching): its own sweep, no batch tables to build
                    old = self._batches.pop(key, None) if self.batched else None
                    if old is not None:
                        st.synchronize()
                        old[1].free()
                    for m in members:
                        self.capi.cpd_als_iter_async(m["h"], m["F"], m["lam"], key[1], m["fit"], stream=st)
        for key in groups:
            cur.wait_stream(self._stream(key))
        n = len(slots)
        if self._fit_dev.numel() < n:
            cap = max(64, 2 * n)
            self._fit_dev = torch.empty(cap, dtype=torch.float64, device="cuda")
            self._fit_host = torch.empty(cap, dtype=torch.float64, pin_memory=True)
        torch.cat([s["fit"] for s in slots], out=self._fit_dev[:n])
        self._fit_host[:n].copy_(self._fit_dev[:n], non_blocking=True)
        self._fit_event.record(cur)
        self._fit_event.synchronize()
        return self._fit_host[:n].tolist()

    def release(self, slot):
        torch = self.torch
        torch.cuda.synchronize()
        res = {"factors": [f.cpu().numpy() for f in slot["F"]], "lambda": slot["lam"].cpu().numpy()}
        old = self._batches.get(slot["key"])
        if old is not None and id(slot["h"]) in old[0]:
            self._batches.pop(slot["key"])[1].free()
        slot["h"].free()
        return res
