"""Continuous-batching server over the komahip request API.

Requests (scanner, phantom, sequence) arrive over time. The scheduler admits
queued requests in arrival order while a slot is free and the request's
device footprint fits the HBM budget; an admitted request copies its phantom
to the device once and keeps phantom and spin state there, and is advanced
by chunks of events on a HIP stream of its own, so chunks of different
requests run on the GPU at the same time. A finished request returns its
signal, releases its device memory and frees its slot for the queue.
Latency is measured from arrival to the signal in host memory.

All device work is in the HIP library; this module only orders calls.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from . import komahip as K


@dataclass
class Job:
    rid: int
    arrival: float  # seconds after the start of the run
    scanner: object
    phantom: object
    seq: object
    tag: str = ""
    spin_steps: int = 0
    footprint: int = 0
    # filled by the server
    admit: float = float("nan")
    finish: float = float("nan")
    status: str = "queued"
    error: str = ""
    signal: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class Server:
    """One context, a pool of streams, at most ``max_slots`` requests in flight."""

    def __init__(self, device: int = 0, precision: str = "mixed", max_slots: int = 8,
                 hbm_budget: Optional[int] = None, chunk_events: int = 1024, keep_signal: bool = False,
                 backend=None):
        """``backend`` = (context, stream factory, event factory) replaces the
        HIP context and torch streams/events (used to test the scheduler on the CPU)."""
        self.max_slots = int(max_slots)
        self.chunk_events = int(chunk_events)
        if backend is None:
            import torch
            self.ctx = K.Context(device, precision, chunk_events=int(chunk_events))
            if hbm_budget is None:
                free, _ = torch.cuda.mem_get_info(device)
                hbm_budget = int(0.8 * free)
            # streams at the default priority
            self.streams = [torch.cuda.Stream(device=device) for _ in range(self.max_slots)]
            self.new_event = torch.cuda.Event
        else:
            self.ctx, make_stream, self.new_event = backend
            self.streams = [make_stream() for _ in range(self.max_slots)]
        self.hbm_budget = int(hbm_budget)
        self.keep_signal = keep_signal
        self.peak_used = 0  # largest sum of admitted footprints seen
        self.peak_active = 0
        self.admit_order = []

    def close(self):
        self.ctx.close()

    def prepare(self, job: Job) -> Job:
        """Fill the job's footprint and grid spin-steps from a host-only plan."""
        info = K.koma_plan_info(job.scanner, job.phantom, job.seq, self.ctx.cfg)
        job.footprint = int(info["footprint"])
        job.spin_steps = int(job.phantom.n) * int(job.seq.n_int)
        return job

    def run(self, jobs, log: Optional[Callable] = None, realtime: bool = True):
        """Serve ``jobs`` (sorted by arrival). With ``realtime`` the arrival times
        are honoured on the wall clock; otherwise everything arrives at once."""
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        queue: deque = deque()
        active = []  # (job, request, stream, event)
        free_streams = list(self.streams)
        used = 0
        done = []
        t0 = time.perf_counter()
        while pending or queue or active:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                queue.append(pending.popleft())
            # admission: arrival order, free slot, footprint within budget
            while queue and len(active) < self.max_slots:
                job = queue[0]
                if job.footprint > self.hbm_budget:
                    queue.popleft()
                    job.status, job.error = "rejected", "footprint exceeds the HBM budget"
                    job.finish = time.perf_counter() - t0
                    done.append(job)
                    continue
                if used + job.footprint > self.hbm_budget:
                    break
                queue.popleft()
                job.admit = time.perf_counter() - t0
                try:
                    req = self.ctx.open(job.scanner, job.phantom, job.seq, "host")
                except K.KomaError as e:  # a bad request fails alone
                    job.status, job.error = "failed", str(e)
                    job.finish = time.perf_counter() - t0
                    done.append(job)
                    continue
                used += job.footprint
                active.append([job, req, free_streams.pop(), None])
                self.peak_used = max(self.peak_used, used)
                self.peak_active = max(self.peak_active, len(active))
                self.admit_order.append(job.rid)
            progressed = False
            for slot in list(active):
                job, req, stream, ev = slot
                if ev is not None and not ev.query():
                    continue
                progressed = True
                try:
                    if req.done():
                        sig = req.result(stream)
                        job.finish = time.perf_counter() - t0
                        job.status = "done"
                        if self.keep_signal:
                            job.signal = sig
                        req.close()
                        used -= job.footprint
                        free_streams.append(stream)
                        active.remove(slot)
                        done.append(job)
                        continue
                    req.advance(self.chunk_events, stream)
                    ev = self.new_event()
                    ev.record(stream)
                    slot[3] = ev
                except K.KomaError as e:
                    job.status, job.error = "failed", str(e)
                    job.finish = time.perf_counter() - t0
                    req.close()
                    used -= job.footprint
                    free_streams.append(stream)
                    active.remove(slot)
                    done.append(job)
            if not progressed:
                time.sleep(20e-6)
        if log:
            log(f"[serve] {len(done)} requests in {time.perf_counter() - t0:.3f} s")
        return done


def summarize(jobs, wall: float) -> dict:
    ok = [j for j in jobs if j.status == "done"]
    lat = np.array([j.latency for j in ok]) * 1e3
    steps = sum(j.spin_steps for j in ok)
    return {"n_done": len(ok), "n_failed": len(jobs) - len(ok),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_ms": float(lat.mean()) if len(lat) else None,
            "throughput_req_s": len(ok) / wall if wall > 0 else None,
            "gspin_steps_per_s": steps / wall / 1e9 if wall > 0 else None}


def make_jobs(n: int, seed: int, scale: float, lo: float = 3.0, hi: float = 6.0, warm: int = 0):
    """Seeded request stream (sizes log-uniform in [10^lo, 10^hi] spins, GRE /
    EPI / one SE-EPI slice, Poisson arrivals with mean gap ``scale`` s)."""
    from . import workloads as W
    reqs = W.serving_requests(n + warm, seed, lo, hi)
    sc = W.Scanner()
    jobs = []
    for r in reqs:
        jobs.append(Job(r.rid, r.arrival * scale, sc, W.serving_phantom(r), W.serving_sequence(r.kind),
                        tag=f"{r.kind}:{r.n_spins}"))
    return jobs[:warm], jobs[warm:]


def benchmark(ctx_device: int = 0, n_requests: int = 200, rho: float = 0.8, seed: int = 3000,
              max_slots: int = 8, log=None) -> dict:
    """Serving figures: the service capacity of FIFO one-at-a-time, then the
    same Poisson stream at load ``rho`` of that capacity served FIFO and with
    continuous batching."""
    import torch
    srv1 = Server(ctx_device, "mixed", max_slots=1)
    warm, jobs = make_jobs(n_requests, seed, 1.0, warm=10)  # unit-mean gaps, scaled below
    for j in warm + jobs:
        srv1.prepare(j)
    srv1.run(warm, realtime=False)
    # saturated FIFO capacity: everything queued at t = 0
    arrivals = [j.arrival for j in jobs]
    t = time.perf_counter()
    srv1.run(jobs, realtime=False)
    torch.cuda.synchronize()
    t_fifo_sat = time.perf_counter() - t
    mu = len(jobs) / t_fifo_sat  # requests/s one at a time
    gap = 1.0 / (rho * mu)
    t_first = arrivals[0]
    for j, a in zip(jobs, arrivals):
        j.arrival = (a - t_first) * gap
        j.admit = j.finish = float("nan")
        j.status = "queued"
    out = {"requests": len(jobs), "rho_of_fifo_capacity": rho, "fifo_capacity_req_s": mu,
           "arrival_rate_req_s": rho * mu, "max_slots": max_slots}
    t = time.perf_counter()
    res = srv1.run(jobs, realtime=True)
    out["fifo"] = summarize(res, time.perf_counter() - t)
    srv1.close()
    for j in jobs:
        j.admit = j.finish = float("nan")
        j.status = "queued"
    srv = Server(ctx_device, "mixed", max_slots=max_slots)
    srv.run(warm, realtime=False)
    t = time.perf_counter()
    res = srv.run(jobs, realtime=True)
    out["batched"] = summarize(res, time.perf_counter() - t)
    # saturated throughput of the batched server (everything queued at t = 0)
    for j in jobs:
        j.arrival = 0.0
        j.admit = j.finish = float("nan")
        j.status = "queued"
    t = time.perf_counter()
    res = srv.run(jobs, realtime=False)
    out["batched_saturated"] = summarize(res, time.perf_counter() - t)
    srv.close()
    out["p50_ms"] = out["batched"]["p50_ms"]
    out["p99_ms"] = out["batched"]["p99_ms"]
    if log:
        log(f"[serve] FIFO capacity {mu:.1f} req/s; at rho={rho}: FIFO p50/p99 "
            f"{out['fifo']['p50_ms']:.2f}/{out['fifo']['p99_ms']:.2f} ms, batched "
            f"{out['p50_ms']:.2f}/{out['p99_ms']:.2f} ms; saturated batched "
            f"{out['batched_saturated']['throughput_req_s']:.1f} req/s")
    return out
