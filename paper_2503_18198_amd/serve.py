"""Continuous-batching CP-ALS server.

Jobs (a sparse tensor, a rank, a stopping rule) arrive over time.  The loop

* admits waiting jobs in arrival order while a slot is free and their device
  footprint (the N mode copies, workspace, factors; ``mttkrp_footprint``)
  fits in what is left of the HBM budget; state then stays on the device;
* groups the active jobs by the executor's group key ((N, R) on the GPU, so
  a group's per-mode MTTKRPs share one launch pair through
  ``cpd_als_batch_iter_async``) and keeps at most one sweep of each group in
  flight: a group whose sweep has completed is stepped again at once, without
  waiting for slower groups;
* when a group's sweep completes, reads its jobs' fits, retires jobs whose fit
  changed by less than ``tol`` or that reached ``max_iters``, releases their
  memory and admits waiting jobs into the freed room.

Requests that arrive while others run are admitted at once and join their
group's next sweep, so new and old jobs share the GPU.  With
``build_threads`` > 0 a job's device state (its layout build and initial
factors) is made on a worker thread, so it overlaps the sweeps in flight; memory is
reserved when the job is admitted, in arrival order.  A tensor's results do
not depend on which other jobs share its sweeps: the batched sweep is bitwise
the single-tensor sweep.

The executor is an interface so the scheduling logic can be tested on the
CPU with a fake one.  Latency = completion time - arrival time.
"""

from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import threading
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

    def build_bytes(self, job: ServeJob) -> int:
        """Transient device bytes admit() holds while it builds the job's state
        (returned to the budget once the build is done)."""
        return 0

    def admit(self, job: ServeJob):
        """Build the job's device state; returns an opaque slot."""
        raise NotImplementedError

    def step(self, slots: Sequence) -> List[float]:
        """One CP-ALS sweep for every slot; returns their fits (in order)."""
        raise NotImplementedError

    def group_key(self, slot):
        """Slots with equal keys are swept together; groups are stepped
        independently.  By default every slot is in one group, so all
        active jobs step in lockstep."""
        return None

    def launch(self, key, slots: Sequence):
        """Start one sweep of one group's slots; returns a token for poll().
        The default runs step() to completion."""
        return self.step(slots)

    def poll(self, token) -> Optional[List[float]]:
        """The fits of a launched sweep (in slot order), or None while it runs."""
        return token

    def wait(self, tokens: Sequence, timeout_s: Optional[float]) -> None:
        """Return once one of the launched sweeps has completed or timeout_s
        (None: no limit) has passed.  Default: sweeps complete in launch()."""

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
                 clock: Optional[Callable[[], float]] = None, sleep: Optional[Callable[[float], None]] = None,
                 build_threads: int = 0, on_retire: Optional[Callable[[ServeJob], None]] = None):
        self.ex = executor
        self.on_retire = on_retire
        self.build_threads = int(build_threads)
        self.admit_s = 0.0              # host seconds spent in executor.admit, summed over jobs
        self._admit_lock = threading.Lock()
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.clock = clock or time.monotonic
        self.sleep = sleep or time.sleep
        self.in_use = 0
        self.peak_in_use = 0
        self.steps = 0
        self.log: List[Tuple[float, str, int]] = []

    def _admit(self, job: ServeJob):
        """The job's device state, or the exception that stopped its build
        (a failed build fails that job only)."""
        t = time.perf_counter()
        try:
            slot = self.ex.admit(job)
        except Exception as e:      # noqa: BLE001 - reported as the job's status
            slot = e
        with self._admit_lock:
            self.admit_s += time.perf_counter() - t
        return slot

    def run(self, jobs: Sequence[ServeJob]) -> Dict[str, object]:
        if self.build_threads > 0:
            with concurrent.futures.ThreadPoolExecutor(self.build_threads) as pool:
                return self._run(jobs, pool)
        return self._run(jobs, None)

    def _run(self, jobs: Sequence[ServeJob], pool) -> Dict[str, object]:
        pending = sorted(jobs, key=lambda j: (j.arrival_s, j.job_id))
        waiting: List[ServeJob] = []
        ready: Dict[object, List[Tuple[ServeJob, object]]] = {}     # group -> members between sweeps
        flight: Dict[object, Tuple[object, List[Tuple[ServeJob, object]]]] = {}   # group -> (token, members)
        building: List[Tuple[ServeJob, concurrent.futures.Future]] = []
        n_active = 0
        done: List[ServeJob] = []
        t0 = self.clock()
        pi = 0

        def built(job: ServeJob, slot):
            """A build has ended: hand back its transient bytes; a failed one
            also hands back the job's reservation and slot."""
            nonlocal n_active
            self.in_use -= self.ex.build_bytes(job)
            if isinstance(slot, Exception):
                self.in_use -= self.ex.footprint(job)
                n_active -= 1
                job.status = f"failed: build: {slot}"
                job.finished_s = self.clock() - t0
                done.append(job)
                self.log.append((job.finished_s, "fail", job.job_id))
                return
            ready.setdefault(self.ex.group_key(slot), []).append((job, slot))

        while pi < len(pending) or waiting or n_active:
            now = self.clock() - t0
            while pi < len(pending) and pending[pi].arrival_s <= now:
                waiting.append(pending[pi])
                pi += 1
            # admission in arrival order, by slot and by memory
            while waiting and n_active < self.max_slots:
                job = waiting[0]
                need = self.ex.footprint(job) + self.ex.build_bytes(job)
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
                self.in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                n_active += 1
                job.status = "running"
                if pool is not None:
                    job.admitted_s = self.clock() - t0
                    self.log.append((job.admitted_s, "admit", job.job_id))
                    building.append((job, pool.submit(self._admit, job)))
                else:
                    slot = self._admit(job)
                    job.admitted_s = self.clock() - t0
                    self.log.append((job.admitted_s, "admit", job.job_id))
                    built(job, slot)
            if building:
                still_building = []
                for job, fut in building:
                    if fut.done():
                        built(job, fut.result())
                    else:
                        still_building.append((job, fut))
                building = still_building
            if not n_active:
                if pi < len(pending):
                    self.sleep(max(0.0, pending[pi].arrival_s - (self.clock() - t0)))
                continue
            # every group with no sweep in flight starts its next one
            for key in [k for k in ready if k not in flight]:
                members = ready.pop(key)
                flight[key] = (self.ex.launch(key, [s for _, s in members]), members)
                self.steps += 1
            completed = False
            for key in list(flight):
                token, members = flight[key]
                fits = self.ex.poll(token)
                if fits is None:
                    continue
                del flight[key]
                completed = True
                still = []
                for (job, slot), f in zip(members, fits):
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
                        n_active -= 1
                        job.finished_s = self.clock() - t0
                        done.append(job)
                        self.log.append((job.finished_s, "retire", job.job_id))
                        if self.on_retire is not None:
                            self.on_retire(job)
                    else:
                        still.append((job, slot))
                if still:
                    # survivors keep their order ahead of jobs admitted meanwhile
                    ready[key] = still + ready.get(key, [])
            if not completed and (flight or building):
                timeout = pending[pi].arrival_s - (self.clock() - t0) if pi < len(pending) else None
                timeout = None if timeout is None else max(0.0, timeout)
                if flight:
                    if building:
                        # builds finish on their own threads: look at them every 0.2 ms
                        timeout = 2e-4 if timeout is None else min(timeout, 2e-4)
                    self.ex.wait([t for t, _ in flight.values()], timeout)
                else:
                    concurrent.futures.wait([f for _, f in building], timeout,
                                            return_when=concurrent.futures.FIRST_COMPLETED)
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
            "admit_s_total": self.admit_s,
            "peak_hbm_bytes": self.peak_in_use,
        }


def initial_factors(dims, R: int, seed: int):
    """A job's starting factors: U(0,1) fp32, drawn on the current GPU from
    the job's seed (torch's device generator), one (I_m, R) matrix per mode in
    mode order.  The same seed gives the same bits."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    return [torch.rand((int(d), int(R)), generator=g, device="cuda", dtype=torch.float32) for d in dims]


class GpuExecutor(Executor):
    """Device state per job: layout handle, fp32 factors, lambda and fit on
    the GPU.  Jobs are grouped by (N, R); each group has its own stream and
    runs one batched CP-ALS sweep for two or more members (a lone job runs
    its own sweep, with no batch tables to rebuild).  A job's results are
    bitwise the same either way.  A launched sweep ends with an asynchronous
    copy of the group's fits to pinned host memory and an event; poll()
    queries the event, so groups advance without waiting for each other.

    Layouts and batch tables live in device memory from torch's caching
    allocator (``mttkrp_layout_build_in``, ``mttkrp_batch_create_in``): the
    library neither allocates nor frees it, and memory handed back after a
    job retires is reused in stream order (``record_stream``), so admitting
    and retiring jobs never synchronises the whole device.  The only host
    waits are on one stream: a retiring group's stream before its results are
    read back, and the build's own stream."""

    def __init__(self, batched: bool = True, wide_indices: bool = False):
        import torch

        from . import capi
        self.torch = torch
        self.capi = capi
        self.batched = batched
        # Layout options of every job (wide_indices: 32-bit coordinates in all copies).
        self.opts = dict(wide_indices=int(wide_indices))
        self._batches: Dict[Tuple[int, int], Tuple[tuple, object]] = {}   # group -> (member ids, batch)
        self._groups: Dict[Tuple[int, int], dict] = {}    # group -> stream, event, fit buffers

    def footprint(self, job: ServeJob) -> int:
        lib = self.capi.mttkrp_footprint(job.dims, job.nnz, opts=dict(max_R=job.R, **self.opts))
        return lib + sum(int(d) * job.R * 4 for d in job.dims) + 16 * job.R

    def build_bytes(self, job: ServeJob) -> int:
        return self.capi.mttkrp_build_scratch_bytes(job.dims, job.nnz, opts=dict(max_R=job.R, **self.opts))

    def _bytes(self, n: int):
        # 256-byte aligned by torch's allocator
        return self.torch.empty(max(int(n), 1), dtype=self.torch.uint8, device="cuda")

    def admit(self, job: ServeJob):
        torch = self.torch
        opts = dict(max_R=job.R, **self.opts)
        mem = self._bytes(self.capi.mttkrp_footprint(job.dims, job.nnz, opts=opts))
        nscr = self.capi.mttkrp_build_scratch_bytes(job.dims, job.nnz, opts=opts)
        scratch = self._bytes(nscr) if nscr else None
        h = self.capi.mttkrp_layout_build_in(job.idx, job.val, job.dims, mem, scratch, opts=opts)
        del scratch       # back to torch's cache; the build synchronised its stream
        F = initial_factors(job.dims, job.R, job.seed)
        lam = torch.zeros(job.R, dtype=torch.float64, device="cuda")
        fit = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.capi.cpd_als_init(h, F, job.R)
        return {"job": job, "h": h, "F": F, "lam": lam, "fit": fit, "key": (len(job.dims), job.R)}

    def group_key(self, slot):
        return slot["key"]

    def _group(self, key):
        g = self._groups.get(key)
        if g is None:
            torch = self.torch
            g = {"stream": torch.cuda.Stream(), "event": torch.cuda.Event(),
                 "dev": torch.empty(0, dtype=torch.float64, device="cuda"),
                 "host": torch.empty(0, dtype=torch.float64)}
            self._groups[key] = g
        return g

    def launch(self, key, slots):
        torch = self.torch
        g = self._group(key)
        st = g["stream"]
        # factors and state of newly admitted jobs were written on the current stream
        st.wait_stream(torch.cuda.current_stream())
        for m in slots:
            if not m.get("recorded"):
                # memory made on another stream, used on the group's: reused only after the group's work
                for t in [m["h"].dev_mem, m["lam"], m["fit"], *m["F"]]:
                    t.record_stream(st)
                m["recorded"] = True
        with torch.cuda.stream(st):
            if self.batched and len(slots) > 1:
                ids = tuple(id(m["h"]) for m in slots)
                old = self._batches.get(key)
                if old is None or old[0] != ids:
                    if old is not None:
                        old[1].free()      # host state only; its memory returns to torch's cache
                    hs = [m["h"] for m in slots]
                    mem = self._bytes(self.capi.mttkrp_batch_bytes(hs, key[1]))
                    self._batches[key] = (ids, self.capi.mttkrp_batch_create_in(hs, key[1], mem, stream=st))
                b = self._batches[key][1]
                self.capi.cpd_als_batch_iter_async(b, [m["F"] for m in slots], [m["lam"] for m in slots],
                                                   [m["fit"] for m in slots], stream=st)
            else:
                # one job (or no batching): its own sweep, no batch tables to build
                old = self._batches.pop(key, None) if self.batched else None
                if old is not None:
                    old[1].free()
                for m in slots:
                    self.capi.cpd_als_iter_async(m["h"], m["F"], m["lam"], key[1], m["fit"], stream=st)
            n = len(slots)
            if g["dev"].numel() < n:
                # the buffers are idle here: the group has no other sweep in flight
                cap = max(16, 2 * n)
                g["dev"] = torch.empty(cap, dtype=torch.float64, device="cuda")
                g["host"] = torch.empty(cap, dtype=torch.float64, pin_memory=True)
            torch.cat([s["fit"] for s in slots], out=g["dev"][:n])
            g["host"][:n].copy_(g["dev"][:n], non_blocking=True)
            g["event"].record(st)
        return (key, n)

    def poll(self, token):
        key, n = token
        g = self._groups[key]
        if not g["event"].query():
            return None
        return g["host"][:n].tolist()

    def wait(self, tokens, timeout_s):
        end = None if timeout_s is None else time.monotonic() + timeout_s
        events = [self._groups[key]["event"] for key, _ in tokens]
        while not any(e.query() for e in events):
            if end is not None and time.monotonic() >= end:
                return

    def step(self, slots):
        order: Dict[Tuple[int, int], list] = {}
        for i, s in enumerate(slots):
            order.setdefault(s["key"], []).append(i)
        tokens = {key: self.launch(key, [slots[i] for i in idx]) for key, idx in order.items()}
        fits = [0.0] * len(slots)
        for key, idx in order.items():
            self._groups[key]["event"].synchronize()
            for i, f in zip(idx, self.poll(tokens[key])):
                fits[i] = f
        return fits

    def release(self, slot):
        torch = self.torch
        st = self._group(slot["key"])["stream"]
        st.synchronize()
        with torch.cuda.stream(st):
            res = {"factors": [f.cpu().numpy() for f in slot["F"]], "lambda": slot["lam"].cpu().numpy()}
        old = self._batches.get(slot["key"])
        if old is not None and id(slot["h"]) in old[0]:
            self._batches.pop(slot["key"])[1].free()
        slot["h"].free()
        return res
