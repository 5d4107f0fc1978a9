"""koma_simulate_async: the same results as koma_simulate when calls are
pipelined (the host packs the next simulation while the device runs the
previous one), scratch reuse ordered across calls of different sizes and
across streams, and device-side phantom validation reported through the
status word with the outputs left untouched."""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W
from tests._gpu import case, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2301_02702_amd import komahip
    komahip.lib()
    return komahip


def _sig(torch, ph, seq):
    n_sig = max(getattr(ph, "n_coils", 0) or 0, 1)
    shape = (n_sig, ph.n_groups, seq.n_adc, 2) if n_sig > 1 else (ph.n_groups, seq.n_adc, 2)
    return torch.full(shape, -7.0, dtype=torch.float64, device="cuda:0")


def _z(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pipelined_calls_match_synchronous_ones(K, prec):
    """Eight queued calls alternating a small and a larger case (so the
    scratch grows while earlier work is queued), one synchronisation at the
    end: every output equals the synchronous call's bit for bit."""
    import torch
    ctx = K.Context(0, prec)
    try:
        cases = [case("epi_small"), case("gre"), (W.Scanner(),) + (W.with_coils(case("epi_small")[1], 3),
                                                                    case("epi_small")[2])]
        ref = []
        for sc, ph, seq in cases:
            dph = K.device_phantom(ph)
            ref.append(_z(ctx.simulate(sc, dph, seq, where="device", sig=_sig(torch, ph, seq))))
        stream = torch.cuda.current_stream()
        outs, keep = [], []
        for k in range(8):
            sc, ph, seq = cases[k % len(cases)]
            dph = K.device_phantom(ph)
            sig = _sig(torch, ph, seq)
            st = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
            ctx.simulate_async(sc, dph, seq, sig, stream=stream, status=st)
            outs.append((k % len(cases), sig, st))
            keep.append(dph)
        torch.cuda.synchronize()
        for i, sig, st in outs:
            assert int(st.cpu()[0]) == 0
            assert np.array_equal(_z(sig), ref[i]), i
        say(f"[async] {prec}: 8 pipelined calls identical to the synchronous ones")
    finally:
        ctx.close()


def test_async_then_sync_on_other_streams(K):
    """Queued work on a side stream, then a synchronous call on the
    context's own stream: the second call waits for the first (shared
    scratch), and both results are right."""
    import torch
    ctx = K.Context(0, "mixed")
    try:
        sc, ph, seq = case("epi_small")
        dph = K.device_phantom(ph)
        ref = _z(ctx.simulate(sc, dph, seq, where="device", sig=_sig(torch, ph, seq)))
        side = torch.cuda.Stream()
        a = _sig(torch, ph, seq)
        with torch.cuda.stream(side):
            ctx.simulate_async(sc, dph, seq, a, stream=side)
        b = ctx.simulate(sc, dph, seq, where="device", sig=_sig(torch, ph, seq))
        side.synchronize()
        assert np.array_equal(_z(a), ref) and np.array_equal(_z(b), ref)
    finally:
        ctx.close()


def test_invalid_device_phantom_sets_status_and_leaves_outputs(K):
    import torch
    ctx = K.Context(0, "mixed")
    try:
        sc, ph, seq = case("epi_small")
        dph = K.device_phantom(ph)
        dph["x"][5] = float("nan")
        dph["pd"][7] = -1.0
        sig = _sig(torch, ph, seq)
        st = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        ctx.simulate_async(sc, dph, seq, sig, status=st)
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == 1 | 2
        assert bool(torch.all(sig == -7.0))
        # host-side errors are reported at once, and nothing is queued
        bad = W.Sequence(seq.t[::-1].copy(), seq.gx, seq.gy, seq.gz, seq.b1, seq.adc_idx)
        with pytest.raises(K.KomaError):
            ctx.simulate_async(sc, K.device_phantom(ph), bad, _sig(torch, ph, seq))
    finally:
        ctx.close()


def test_validation_word_is_cleared_for_every_call(K):
    """The phantom-check word is zeroed by each call's upload: a valid call
    right after an invalid one (queued behind it, and synchronous) reports 0
    and writes its outputs, bit for bit the reference."""
    import torch
    ctx = K.Context(0, "mixed")
    try:
        sc, ph, seq = case("epi_small")
        good = K.device_phantom(ph)
        ref = _z(ctx.simulate(sc, good, seq, where="device", sig=_sig(torch, ph, seq)))
        bad = K.device_phantom(ph)
        bad["t1"][3] = -1.0
        outs = []
        for dph in (bad, good, bad, good):
            sig = _sig(torch, ph, seq)
            st = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
            ctx.simulate_async(sc, dph, seq, sig, status=st)
            outs.append((sig, st))
        torch.cuda.synchronize()
        for k, (sig, st) in enumerate(outs):
            if k % 2 == 0:
                assert int(st.cpu()[0]) == 4 and bool(torch.all(sig == -7.0)), k
            else:
                assert int(st.cpu()[0]) == 0 and np.array_equal(_z(sig), ref), k
        with pytest.raises(K.KomaError):
            ctx.simulate(sc, bad, seq, where="device", sig=_sig(torch, ph, seq))
        assert np.array_equal(_z(ctx.simulate(sc, good, seq, where="device", sig=_sig(torch, ph, seq))), ref)
    finally:
        ctx.close()
