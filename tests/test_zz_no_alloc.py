"""koma_simulate_noalloc: the simulation of koma_simulate_async in the
library's static device scratch, with no allocation. Through the C ABI, its
outputs are checked against koma_simulate_async's on the same inputs, at the
parity bar of each form (FP64 1e-10, mixed 1e-4, per signal row, normalised
by the row's max), on two calls in a row, the second with a smaller input
(the static scratch keeps the first call's contents); the final state and
the status word too; a simulation too large for the scratch is refused
before any device work, outputs untouched."""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W
from tests._gpu import case, check, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2301_02702_amd import komahip
    komahip.lib()
    return komahip


def _sig(torch, ph, seq):
    return torch.full((ph.n_groups, seq.n_adc, 2), -7.0, dtype=torch.float64, device="cuda:0")


def _z(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def _small():
    """A smaller second input: a ragged subset of the EPI phantom on a short
    random grid with excitation, precession and ADC samples, in two groups."""
    rng = np.random.default_rng(77)
    sc, ph, _ = case("epi_small")
    sub = ph.subset(np.arange(0, 1500, 3))  # 500 spins: 7 full tiles + 52 lanes
    sub.group_off = np.array([0, 210, sub.n], dtype=np.int64)
    seq = W.random_sequence(rng, 300, p_rf=0.3, p_adc=0.5)
    return sc, sub, seq


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_async_on_two_calls(K, prec):
    import torch
    ctx = K.Context(0, prec)
    try:
        cap = K.lib().koma_noalloc_capacity()
        assert cap == 64 << 20
        stream = torch.cuda.current_stream()
        for label, (sc, ph, seq), with_m in (("epi_small", case("epi_small"), True), ("small", _small(), False)):
            say(f"[noalloc] {prec} {label}: {ph.n} spins x {seq.n_int} intervals, {seq.n_adc} ADC")
            dph = K.device_phantom(ph)
            ref = _sig(torch, ph, seq)
            ref_m = torch.zeros((ph.n, 3), dtype=torch.float64, device="cuda:0") if with_m else None
            ctx.simulate_async(sc, dph, seq, ref, stream=stream, m_final=ref_m)
            got = _sig(torch, ph, seq)
            got_m = torch.zeros((ph.n, 3), dtype=torch.float64, device="cuda:0") if with_m else None
            st = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
            ctx.simulate_noalloc(sc, dph, seq, got, stream=stream, m_final=got_m, status=st)
            torch.cuda.synchronize()
            assert int(st.cpu()[0]) == 0
            a, b = _z(got), _z(ref)
            check(a, b, prec, f"noalloc vs async, {label}")
            say(f"[noalloc] {prec} {label}: bitwise equal to async: {np.array_equal(a, b)}")
            if with_m:
                mg, mr = got_m.cpu().numpy(), ref_m.cpu().numpy()
                tol = 1e-10 if prec == "fp64" else 1e-4
                assert np.max(np.abs(mg - mr)) <= tol * max(float(np.max(np.abs(mr))), 1e-300)
    finally:
        ctx.close()


def test_noalloc_refuses_a_simulation_beyond_its_scratch(K):
    """The full-size EPI phantom tiled 32 times (2.1e6 spins) in the FP64
    form with its final state: its snapshots and spin state alone exceed the
    static scratch, so the call fails with KOMA_E_BUDGET before any device
    work, outputs untouched; a call that fits then still works."""
    import torch
    ctx = K.Context(0, "fp64")
    try:
        sc, ph, seq = case("epi")
        big = W.Phantom(np.tile(ph.x, 32), np.tile(ph.y, 32), np.tile(ph.z, 32), np.tile(ph.pd, 32),
                        np.tile(ph.t1, 32), np.tile(ph.t2, 32), np.tile(ph.dw, 32))
        dph = K.device_phantom(big)
        sig = _sig(torch, big, seq)
        m = torch.full((big.n, 3), -3.0, dtype=torch.float64, device="cuda:0")
        with pytest.raises(K.KomaError) as ei:
            ctx.simulate_noalloc(sc, dph, seq, sig, m_final=m)
        assert ei.value.status == -5  # KOMA_E_BUDGET
        say(f"[noalloc] refused: {ei.value}")
        torch.cuda.synchronize()
        assert bool(torch.all(sig == -7.0)) and bool(torch.all(m == -3.0))
        sc, ph, seq = _small()
        dph = K.device_phantom(ph)
        ref = _sig(torch, ph, seq)
        ctx.simulate_async(sc, dph, seq, ref)
        got = _sig(torch, ph, seq)
        ctx.simulate_noalloc(sc, dph, seq, got)
        torch.cuda.synchronize()
        check(_z(got), _z(ref), "fp64", "noalloc vs async after a refusal")
    finally:
        ctx.close()
