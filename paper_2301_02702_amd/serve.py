"""Continuous-batching server over the komahip request API.

Requests (scanner, phantom, sequence) arrive over time. The scheduler admits
queued requests while a slot is free and the request's device footprint fits
the HBM budget beside the bytes the open requests hold; an admitted request
copies its phantom to the device once and keeps phantom and spin state
there, and is advanced by chunks of events on a HIP stream of its own, so
chunks of different requests run on the GPU at the same time. A finished
request returns its signal, releases its device memory and frees its slot
for the queue. Latency is measured from arrival to the signal in host
memory.

Admission order: ``fifo`` takes the queue in arrival order (the head waits
until it fits); ``small_first`` takes the queued request with the least work
(spins x intervals) that fits, unless the oldest one has waited longer than
``max_wait`` seconds, which then goes first (no starvation).

All device work is in the HIP library; this module only orders calls. The
library also enforces the budget on the memory it really holds (cached
blocks of closed requests included).
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
                 backend=None, policy: str = "fifo", max_wait: float = 0.05):
        """``backend`` = (context, stream factory, event factory) replaces the
        HIP context and torch streams/events (used to test the scheduler on the CPU)."""
        self.max_slots = int(max_slots)
        self.chunk_events = int(chunk_events)
        if policy not in ("fifo", "small_first"):
            raise ValueError(policy)
        self.policy = policy
        self.max_wait = float(max_wait)
        if backend is None:
            import torch
            if hbm_budget is None:
                free, _ = torch.cuda.mem_get_info(device)
                hbm_budget = int(0.8 * free)
            self.ctx = K.Context(device, precision, chunk_events=int(chunk_events), hbm_budget=int(hbm_budget))
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

    def _held(self, used: int) -> int:
        """Device bytes the open requests hold: the library's count where the
        context reports one, else the sum of admitted footprints."""
        mem = getattr(self.ctx, "mem", None)
        return max(used, mem()["held"]) if mem else used

    def _next(self, queue, now: float, used: int):
        """Index in ``queue`` of the request to admit now, or None."""
        held = self._held(used)
        if self.policy == "fifo" or now - queue[0].arrival > self.max_wait:
            return 0 if held + queue[0].footprint <= self.hbm_budget else None
        best = None
        for i, j in enumerate(queue):
            if held + j.footprint <= self.hbm_budget and (best is None or j.spin_steps < queue[best].spin_steps):
                best = i
        return best

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
            # requests that can never fit are rejected on arrival
            for job in [j for j in queue if j.footprint > self.hbm_budget]:
                queue.remove(job)
                job.status, job.error = "rejected", "footprint exceeds the HBM budget"
                job.finish = time.perf_counter() - t0
                done.append(job)
            # admission: free slot, footprint within budget, in policy order
            while queue and len(active) < self.max_slots:
                k = self._next(queue, now, used)
                if k is None:
                    break
                job = queue[k]
                del queue[k]
                job.admit = time.perf_counter() - t0
                try:
                    req = self.ctx.open(job.scanner, job.phantom, job.seq, "host")
                except K.KomaError as e:
                    if e.status == K.KOMA_E_BUDGET and active:
                        # the device memory the open requests hold (their blocks
                        # may be larger than their footprints) leaves no room
                        # now: the request waits for one of them to finish
                        queue.insert(k, job)
                        break
                    job.status, job.error = "failed", str(e)  # a bad request fails alone
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


def _reset(jobs, arrivals=None):
    for k, j in enumerate(jobs):
        if arrivals is not None:
            j.arrival = arrivals[k]
        j.admit = j.finish = float("nan")
        j.status = "queued"
        j.error = ""


def benchmark(ctx_device: int = 0, n_requests: int = 1000, n_warm: int = 50, rhos=(0.5, 0.8, 0.95),
              seed: int = 3000, max_slots: int = 8, forced_budget: int = 256 << 20, log=None) -> dict:
    """Serving figures on one seeded stream of ``n_requests`` requests (after
    ``n_warm`` warm-up requests): the saturated capacity mu (requests/s with
    every request queued at t = 0) of the batched server and of FIFO one at a
    time; then Poisson arrivals at rate rho * mu(batched) for every rho,
    served by continuous batching (arrival order and small-first) and by FIFO;
    and the batched server at rho = 0.8 under a forced HBM budget."""
    import torch
    warm, jobs = make_jobs(n_requests, seed, 1.0, warm=n_warm)  # unit-mean gaps, scaled below
    unit = [j.arrival - jobs[0].arrival for j in jobs]
    servers = {"batched": Server(ctx_device, "mixed", max_slots=max_slots),
               "small_first": Server(ctx_device, "mixed", max_slots=max_slots, policy="small_first"),
               "fifo": Server(ctx_device, "mixed", max_slots=1)}
    for j in warm + jobs:
        servers["fifo"].prepare(j)
    for srv in servers.values():
        _reset(warm, [0.0] * len(warm))
        srv.run(warm, realtime=False)
    out = {"requests": len(jobs), "warmup_requests": len(warm), "max_slots": max_slots,
           "spins_per_request": {"min": int(min(j.phantom.n for j in jobs)),
                                 "median": float(np.median([j.phantom.n for j in jobs])),
                                 "max": int(max(j.phantom.n for j in jobs))}}
    cap = {}
    for name in ("batched", "fifo"):
        _reset(jobs, [0.0] * len(jobs))
        t = time.perf_counter()
        res = servers[name].run(jobs, realtime=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        cap[name] = len(jobs) / wall
        out[f"saturated_{name}"] = summarize(res, wall)
    mu = cap["batched"]
    out["mu_req_s"] = {"batched": mu, "fifo": cap["fifo"]}
    loads = {}
    for rho in rhos:
        r = {"rho": rho, "arrival_rate_req_s": rho * mu}
        for name in ("batched", "small_first", "fifo"):
            _reset(jobs, [u / (rho * mu) for u in unit])
            t = time.perf_counter()
            res = servers[name].run(jobs, realtime=True)
            r[name] = summarize(res, time.perf_counter() - t)
        loads[str(rho)] = r
        if log:
            log(f"[serve] rho {rho}: batched p50/p99 {r['batched']['p50_ms']:.2f}/{r['batched']['p99_ms']:.2f} ms, "
                f"small-first {r['small_first']['p50_ms']:.2f}/{r['small_first']['p99_ms']:.2f}, "
                f"FIFO {r['fifo']['p50_ms']:.2f}/{r['fifo']['p99_ms']:.2f}")
    out["loads"] = loads
    for srv in servers.values():
        srv.close()
    # a forced budget: requests queue for memory; those larger than it are rejected
    srv = Server(ctx_device, "mixed", max_slots=max_slots, hbm_budget=forced_budget)
    _reset(jobs, [u / (0.8 * mu) for u in unit])
    t = time.perf_counter()
    res = srv.run(jobs, realtime=True)
    fb = summarize(res, time.perf_counter() - t)
    fb.update(budget_bytes=forced_budget, rho=0.8, peak_footprint_sum=srv.peak_used,
              peak_device_bytes=srv.ctx.mem()["peak"],
              rejected=int(sum(j.status == "rejected" for j in res)))
    out["forced_budget"] = fb
    srv.close()
    out["p50_ms"] = loads["0.8"]["batched"]["p50_ms"] if "0.8" in loads else None
    out["p99_ms"] = loads["0.8"]["batched"]["p99_ms"] if "0.8" in loads else None
    if log:
        log(f"[serve] capacity batched {mu:.1f} req/s, FIFO {cap['fifo']:.1f}; forced {forced_budget >> 20} MB "
            f"budget: p50/p99 {fb['p50_ms']:.2f}/{fb['p99_ms']:.2f} ms, {fb['rejected']} rejected, "
            f"peak device bytes {fb['peak_device_bytes']}")
    return out
