"""Serving a stream of independent clustering jobs with continuous batching.

Each job is a whole TPO run (its own graph, attributes and k) through the
C ABI.  Up to `workers` jobs run at once, each on its own HIP stream: one
host thread per stream calls tpo_execute, which returns when its job is
done (ctypes releases the interpreter lock for the call), so the GPU
overlaps the jobs' kernels (each job keeps to its own stream: the plans are
made with one_stream, so no job opens a second stream of its own).  A job is admitted, in arrival order, as soon as
a worker is free and its workspace fits in the HBM budget.  The budget is one
device buffer allocated when serving starts; each job's workspace is carved
out of it at admission (first fit, 256-byte aligned) and returned when the
job ends, so serving makes no device allocation per job.  Every kernel is
deterministic, so a job's result does not depend on what runs beside it.

The subspace-iteration kernel synchronises its workgroups with a grid
barrier, so all of its workgroups (ceil(N / 16), at most 256 and at most one
per CU, for the N x N Gram it iterates on) must be resident at once.  Admission therefore also
keeps the barrier workgroups of the jobs in flight within the 256 CUs (one
CU each at most), whatever the number of workers.

Resident graphs: jobs that name the same graph (Job.graph_key) and the same
parameters reuse one workspace, which keeps the graph's CSR, degrees and hub
lists in HBM between jobs: the first job ingests the edge list, later ones
run tpo_execute_resident and skip ingest.  A resident workspace is held while
idle and given back, least recently used first, when a new job needs the
memory.  A job whose graph's workspace is busy with another job runs on a
workspace of its own (and ingests).
"""
from __future__ import annotations

import queue
import threading
import time
from dataclasses import dataclass, field

import paper_2405_11922_amd as tpo

MAX_WORKERS = 16
BARRIER_CUS = 256  # CUs of one MI355X


def barrier_workgroups(plan, d_u: int) -> int:
    """Workgroups of the plan's widest subspace-iteration launch: the
    reduction's (N = d_U, when it reduces) and the embedding's (N = 2 d_eff)."""
    d_eff, l_r, _ = tpo.tpo_plan_dims(plan)
    n_red = d_u if l_r > 0 else 0
    return min(BARRIER_CUS, max((n_red + 15) // 16, (2 * d_eff + 15) // 16))


@dataclass
class Job:
    """One clustering request: device tensors plus the method parameters
    (those of tpo_plan_create).  `arrival` is seconds after the stream
    starts."""

    job_id: int
    arrival: float
    edge_u: object
    edge_v: object
    x_u: object
    n_v: int
    params: dict
    edge_w: object = None
    graph_key: object = None  # jobs with equal keys share one edge list


@dataclass
class Result:
    job_id: int
    arrival: float
    admitted: float
    done: float
    labels: object = None
    objective: tuple = (0.0, 0.0)
    workspace_bytes: int = 0
    error: str = ""
    started: float = 0.0  # the worker took the job
    exec_s: float = 0.0   # inside tpo_execute
    resident: bool = False  # ran on its graph's resident workspace (no ingest)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Pool:
    """First-fit sub-allocation of one device buffer (offsets 256-byte
    aligned); callers hold the server's lock."""

    def __init__(self, nbytes: int):
        self.free = [(0, nbytes)]  # (offset, size), sorted by offset

    def take(self, nbytes: int):
        need = (nbytes + 255) & ~255
        for i, (off, size) in enumerate(self.free):
            if size >= need:
                if size == need:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + need, size - need)
                return off
        return None

    def give(self, off: int, nbytes: int):
        need = (nbytes + 255) & ~255
        self.free.append((off, need))
        self.free.sort()
        merged = []
        for o, sz in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + sz)
            else:
                merged.append((o, sz))
        self.free = merged


@dataclass
class _Slot:
    """A resident workspace: a plan and its pool region, holding one graph."""

    plan: int
    off: int
    nbytes: int
    busy: bool = False
    ingested: bool = False
    last_used: float = 0.0


@dataclass
class Server:
    device: object = "cuda:0"
    hbm_budget: int = 64 << 30  # bytes of workspace (in flight and resident) at most
    workers: int = MAX_WORKERS
    resident: bool = True  # keep each graph's workspace (and CSR) between its jobs
    _lock: threading.Condition = field(default_factory=threading.Condition, init=False)
    _in_flight: int = field(default=0, init=False)
    _busy: int = field(default=0, init=False)
    _barrier_wg: int = field(default=0, init=False)

    def _plan(self, job: Job):
        x = job.x_u
        n_u, d_u = x.shape
        xdt = tpo._TORCH_XDT.get(str(x.dtype), "f32")
        h = tpo.tpo_plan_create(n_u, job.n_v, job.edge_u.numel(), d_u, weighted=job.edge_w is not None,
                                x_dtype=xdt, one_stream=True, **job.params)
        return h, tpo.tpo_plan_workspace_bytes(h), barrier_workgroups(h, d_u)

    @staticmethod
    def _slot_key(job: Job):
        if job.graph_key is None:
            return None
        return (job.graph_key, str(job.x_u.dtype), tuple(sorted(job.params.items())))

    def _take(self, nbytes: int):
        """A pool region, evicting idle resident workspaces (least recently
        used first) while the pool is short; None if that does not free
        enough.  Holds the lock."""
        while True:
            off = self._pool.take(nbytes)
            if off is not None:
                return off
            idle = [(sl.last_used, key) for key, sl in self._slots.items() if not sl.busy]
            if not idle:
                return None
            _, key = min(idle, key=lambda t: t[0])
            sl = self._slots.pop(key)
            self._pool.give(sl.off, sl.nbytes)
            tpo.tpo_plan_destroy(sl.plan)

    def _worker(self, q: "queue.Queue", results: list, t0: float):
        import torch

        stream = torch.cuda.Stream(device=self.device)
        while True:
            item = q.get()
            if item is None:
                return
            job, h, nbytes, wg, off, admitted, slot = item
            res = Result(job.job_id, job.arrival, admitted, 0.0, workspace_bytes=nbytes)
            res.started = time.perf_counter() - t0
            ok = False
            try:
                with torch.cuda.stream(stream):
                    wsv = self._buf[off: off + nbytes]
                    labels = torch.empty(job.x_u.shape[0], dtype=torch.int32, device=self.device)
                    e0 = time.perf_counter()
                    if slot is not None and slot.ingested:
                        res.objective = tpo.tpo_execute_resident(h, job.x_u, wsv, labels, stream=stream.cuda_stream)
                        res.resident = True
                    else:
                        res.objective = tpo.tpo_execute(h, job.edge_u, job.edge_v, job.x_u, wsv, labels,
                                                        edge_w=job.edge_w, stream=stream.cuda_stream)
                    res.exec_s = time.perf_counter() - e0
                    res.labels = labels
                    ok = True
            except tpo.TpoError as e:
                res.error = str(e)
            finally:
                res.done = time.perf_counter() - t0
                with self._lock:
                    if slot is not None:
                        slot.busy = False
                        slot.ingested = slot.ingested or ok
                        slot.last_used = res.done
                    else:
                        tpo.tpo_plan_destroy(h)
                        self._pool.give(off, nbytes)
                    self._in_flight -= nbytes
                    self._barrier_wg -= wg
                    self._busy -= 1
                    results.append(res)
                    self._lock.notify_all()

    def run(self, jobs: list, realtime: bool = True) -> list:
        """Serves `jobs` (sorted by arrival).  realtime: wait for each job's
        arrival time; otherwise all jobs are present at time 0.  Returns the
        results in completion order."""
        if not 1 <= self.workers <= MAX_WORKERS:
            raise ValueError(f"workers must be in 1..{MAX_WORKERS}")
        import torch

        q: "queue.Queue" = queue.Queue()
        results: list = []
        self._buf = torch.empty(self.hbm_budget, dtype=torch.uint8, device=self.device)
        assert self._buf.data_ptr() % 256 == 0
        self._pool = _Pool(self.hbm_budget)
        self._slots = {}
        t0 = time.perf_counter()
        threads = [threading.Thread(target=self._worker, args=(q, results, t0), daemon=True)
                   for _ in range(self.workers)]
        for t in threads:
            t.start()
        try:
            for job in sorted(jobs, key=lambda j: j.arrival):
                if realtime:
                    wait = job.arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                key = self._slot_key(job) if self.resident else None
                h, nbytes, wg = self._plan(job)
                if nbytes > self.hbm_budget:
                    tpo.tpo_plan_destroy(h)
                    now = time.perf_counter() - t0
                    with self._lock:
                        results.append(Result(job.job_id, job.arrival, now, now,
                                              error="workspace above the HBM budget"))
                    continue
                with self._lock:
                    while True:
                        use, off = None, None
                        if self._busy < self.workers and self._barrier_wg + wg <= BARRIER_CUS:
                            slot = self._slots.get(key) if key is not None else None
                            if slot is not None and not slot.busy:
                                # its graph is resident: the slot's plan and workspace
                                tpo.tpo_plan_destroy(h)
                                use, off, h, nbytes = slot, slot.off, slot.plan, slot.nbytes
                                break
                            off = self._take(nbytes)
                            if off is not None:
                                if key is not None and slot is None:
                                    # the first job on this graph: its workspace stays
                                    use = _Slot(h, off, nbytes)
                                    self._slots[key] = use
                                break
                        self._lock.wait()
                    if use is not None:
                        use.busy = True
                    self._busy += 1
                    self._in_flight += nbytes
                    self._barrier_wg += wg
                q.put((job, h, nbytes, wg, off, time.perf_counter() - t0, use))
        finally:
            for _ in threads:
                q.put(None)
            for t in threads:
                t.join()
            for sl in self._slots.values():
                tpo.tpo_plan_destroy(sl.plan)
            self._slots = {}
            self._buf = None
        return results


def summarize(results: list) -> dict:
    """jobs/s over the stream and the latency percentiles (arrival to done)."""
    import numpy as np

    ok = [r for r in results if not r.error]
    if not ok:
        return {"jobs": 0, "failed": len(results)}
    lat = np.array([r.latency for r in ok]) * 1e3
    span = max(r.done for r in ok) - min(r.arrival for r in ok)
    wait = np.array([r.started - r.arrival for r in ok]) * 1e3
    exe = np.array([r.exec_s for r in ok]) * 1e3
    return {
        "jobs": len(ok),
        "resident_jobs": sum(1 for r in ok if r.resident),
        "failed": len(results) - len(ok),
        "queue_p50_ms": float(np.percentile(wait, 50)),
        "exec_p50_ms": float(np.percentile(exe, 50)),
        "exec_mean_ms": float(exe.mean()),
        "jobs_per_s": len(ok) / span if span > 0 else None,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "max_ms": float(lat.max()),
    }
