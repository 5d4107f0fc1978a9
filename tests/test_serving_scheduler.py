"""The continuous-batching scheduler on the CPU, with a fake device back end:
arrival-order admission, slot and HBM-budget limits, chunked progress,
failure isolation and rejection of requests larger than the budget."""
import numpy as np

from paper_2301_02702_amd import komahip as K
from paper_2301_02702_amd import serve


class FakeEvent:
    def __init__(self):
        self.polls = 0

    def record(self, stream):
        stream.log.append("record")

    def query(self):  # completes on the second poll
        self.polls += 1
        return self.polls >= 2


class FakeStream:
    def __init__(self):
        self.log = []


class FakeReq:
    def __init__(self, ctx, job_n, chunks):
        self.ctx, self.n, self.left = ctx, job_n, chunks
        ctx.live += 1
        ctx.max_live = max(ctx.max_live, ctx.live)

    def advance(self, n, stream):
        stream.log.append("advance")
        self.left -= 1

    def done(self):
        return self.left <= 0

    def result(self, stream):
        return np.full((1, 4), self.n, dtype=complex)

    def close(self):
        self.ctx.live -= 1


class FakeCtx:
    def __init__(self):
        self.live = 0
        self.max_live = 0

    def open(self, scanner, phantom, seq, where):
        if getattr(phantom, "bad", False):
            raise K.KomaError(-2, "bad phantom")
        return FakeReq(self, phantom.n, chunks=phantom.n % 5 + 1)


class Ph:
    def __init__(self, n, bad=False):
        self.n, self.bad = n, bad


def jobs(sizes, fps, bad=()):
    return [serve.Job(i, 0.0, None, Ph(n, i in bad), None, footprint=f) for i, (n, f) in
            enumerate(zip(sizes, fps))]


def server(slots, budget):
    return serve.Server(max_slots=slots, hbm_budget=budget, keep_signal=True,
                        backend=(FakeCtx(), FakeStream, FakeEvent))


def test_admission_respects_slots_budget_and_arrival_order():
    s = server(3, 100)
    js = jobs(range(10, 22), [30, 50, 20, 40, 10, 60, 25, 25, 25, 5, 70, 30])
    done = s.run(js, realtime=False)
    assert all(j.status == "done" for j in done)
    assert s.peak_used <= 100 and s.ctx.max_live <= 3 and s.peak_active <= 3
    assert s.admit_order == sorted(s.admit_order)  # FIFO admission
    for j in done:
        assert j.signal[0, 0] == j.phantom.n


def test_failures_are_isolated_and_oversized_requests_rejected():
    s = server(2, 100)
    js = jobs([5, 6, 7, 8], [10, 200, 10, 10], bad={2})
    done = {j.rid: j for j in s.run(js, realtime=False)}
    assert done[1].status == "rejected"
    assert done[2].status == "failed" and "bad phantom" in done[2].error
    assert done[0].status == "done" and done[3].status == "done"
    assert s.ctx.live == 0


def test_realtime_arrivals_are_honoured():
    s = server(4, 1000)
    js = jobs([1, 2, 3], [1, 1, 1])
    for j, a in zip(js, (0.0, 0.02, 0.04)):
        j.arrival = a
    done = s.run(js, realtime=True)
    for j in done:
        assert j.admit >= j.arrival - 1e-3 and j.finish >= j.admit


def test_small_first_admits_the_least_work_and_ages_the_oldest():
    s = serve.Server(max_slots=1, hbm_budget=100, keep_signal=True, backend=(FakeCtx(), FakeStream, FakeEvent),
                     policy="small_first", max_wait=1e9)
    js = jobs([10, 11, 12, 13, 14], [10, 10, 10, 10, 10])
    for j, w in zip(js, (50, 40, 30, 20, 10)):
        j.spin_steps = w
    s.run(js, realtime=False)
    assert s.admit_order == [4, 3, 2, 1, 0]  # least work first
    # a request older than max_wait goes first: with max_wait = 0 the order is the arrival order
    s = serve.Server(max_slots=1, hbm_budget=100, keep_signal=True, backend=(FakeCtx(), FakeStream, FakeEvent),
                     policy="small_first", max_wait=0.0)
    js = jobs([10, 11, 12], [10, 10, 10])
    for j, w, a in zip(js, (50, 40, 30), (0.0, 1e-4, 2e-4)):
        j.spin_steps, j.arrival = w, a
    s.run(js, realtime=False)
    assert s.admit_order == [0, 1, 2]


def test_small_first_skips_a_request_that_does_not_fit_yet():
    s = serve.Server(max_slots=4, hbm_budget=100, keep_signal=True, backend=(FakeCtx(), FakeStream, FakeEvent),
                     policy="small_first", max_wait=1e9)
    js = jobs([10, 11, 12], [60, 70, 30])
    for j, w in zip(js, (5, 6, 7)):
        j.spin_steps = w
    done = s.run(js, realtime=False)
    assert all(j.status == "done" for j in done)
    assert s.admit_order[:2] == [0, 2]  # 1 (70) does not fit beside 0 (60); 2 (30) does
    assert s.peak_used <= 100


class TightCtx(FakeCtx):
    """A back end whose device memory per request exceeds the footprint the
    scheduler counts (cached blocks reused at up to twice their size): it
    refuses an open with KOMA_E_BUDGET when the real bytes would not fit."""

    def __init__(self, budget):
        super().__init__()
        self.budget, self.held, self.refused = budget, 0, 0

    def mem(self):
        return {"held": self.held, "cached": 0, "peak": self.held}

    def open(self, scanner, phantom, seq, where):
        real = 2 * phantom.fp
        if self.held + real > self.budget:
            self.refused += 1
            raise K.KomaError(K.KOMA_E_BUDGET, "device memory of open requests would exceed hbm_budget")
        self.held += real
        req = FakeReq(self, phantom.n, chunks=phantom.n % 5 + 1)
        close = req.close

        def release():
            self.held -= real
            close()
        req.close = release
        return req


def test_requests_refused_for_memory_wait_for_it():
    """When the library refuses an open because the memory the open requests
    really hold leaves no room, the request waits for one of them to finish
    (it is not failed), and every request completes."""
    budget = 100
    fps = [30, 20, 25, 40, 10, 35, 15, 45]
    js = []
    for i, f in enumerate(fps):
        ph = Ph(10 + i)
        ph.fp = f
        js.append(serve.Job(i, 0.0, None, ph, None, footprint=f))
    ctx = TightCtx(budget)
    s = serve.Server(max_slots=4, hbm_budget=budget, keep_signal=True, backend=(ctx, FakeStream, FakeEvent))
    done = s.run(js, realtime=False)
    assert all(j.status == "done" for j in done) and len(done) == len(fps)
    assert ctx.refused > 0 and ctx.held == 0
