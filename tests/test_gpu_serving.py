"""Continuous batching on the GPU: every served result matches the FP64
oracle and is the same alone and in the mix, admission respects the HBM
budget, a bad request fails alone."""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W
from tests._gpu import check, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    from paper_2301_02702_amd import komahip, serve
    komahip.lib()
    return serve


def small_jobs(serve, n=16, seed=3100):
    _, jobs = serve.make_jobs(n, seed, 0.0, lo=3.0, hi=4.5)
    return jobs


def test_each_result_is_the_same_alone_and_in_the_mix(serve):
    say("[serving] alone vs mix")
    srv = serve.Server(0, "mixed", max_slots=6, chunk_events=300, keep_signal=True)
    jobs = [srv.prepare(j) for j in small_jobs(serve)]
    done = srv.run(jobs, realtime=False)
    assert all(j.status == "done" for j in done)
    assert srv.peak_active > 1  # requests really overlapped
    import oracle
    for j in done:
        alone = srv.ctx.simulate(j.scanner, j.phantom, j.seq)
        assert np.array_equal(j.signal, alone), j.tag
        ref = oracle.simulate(j.scanner, j.phantom, j.seq, mode=oracle.MODE_BLOCK)
        check(j.signal, ref, "mixed", f"served {j.tag} vs oracle")
    srv.close()


def test_admission_respects_a_small_hbm_budget(serve):
    say("[serving] forced budget")
    probe = serve.Server(0, "mixed", max_slots=8)
    jobs = [probe.prepare(j) for j in small_jobs(serve, 12, 3200)]
    probe.close()
    budget = int(max(j.footprint for j in jobs) * 1.5)
    for policy in ("fifo", "small_first"):
        srv = serve.Server(0, "mixed", max_slots=8, hbm_budget=budget, policy=policy)
        done = srv.run(jobs, realtime=False)
        assert all(j.status == "done" for j in done)
        mem = srv.ctx.mem()
        say(f"[serving] {policy}: budget {budget}, peak footprint sum {srv.peak_used}, "
            f"peak device bytes (held + cached) {mem['peak']}")
        assert srv.peak_used <= budget
        assert mem["peak"] <= budget and mem["held"] == 0  # the memory the library really held
        srv.close()
        for j in jobs:
            j.status, j.admit, j.finish = "queued", float("nan"), float("nan")


def test_oversized_and_invalid_requests_fail_alone(serve):
    say("[serving] failure isolation")
    srv = serve.Server(0, "mixed", max_slots=4, keep_signal=True)
    jobs = [srv.prepare(j) for j in small_jobs(serve, 6, 3300)]
    bad = jobs[2]
    bad.phantom = bad.phantom.subset(np.arange(bad.phantom.n))
    bad.phantom.t2[0] = np.nan  # rejected by validation when the request opens
    big = jobs[4]
    big.footprint = srv.hbm_budget + 1  # can never be admitted
    done = {j.rid: j for j in srv.run(jobs, realtime=False)}
    assert done[bad.rid].status == "failed" and "PHANTOM" in done[bad.rid].error
    assert done[big.rid].status == "rejected"
    others = [j for j in jobs if j.rid not in (bad.rid, big.rid)]
    assert all(done[j.rid].status == "done" for j in others)
    srv.close()
