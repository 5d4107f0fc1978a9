"""GPU parity of receive-coil signals against the FP64 oracle.

Coil c's signal is the sum over a group's spins of sens_c * Mxy. The
sample-parallel kernel folds sens_c into each spin's anchor (one grid plane
per coil); the spin-sequential kernel weights every inline sample per coil.
Parity bar as in the static parity tests (tests/_gpu.py): NRMSE and the
largest sample error <= 1e-10 (FP64) and 1e-4 (mixed), per coil and group.
"""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W
from tests._gpu import TOL, case, check, nrmse, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2301_02702_amd import komahip
    komahip.lib()
    return komahip


@pytest.fixture(scope="module")
def ctx(K):
    c = K.Context(0, "mixed")
    yield c
    c.close()


def worst(got, ref):
    return max(float(np.max(nrmse(got[c], ref[c]))) for c in range(ref.shape[0]))


def coil_case(key, n_coils, moving=False):
    sc, ph, seq = case(key)
    ph = W.with_coils(ph, n_coils)
    if moving:
        ph = W.with_velocity(ph, (0.05, 0.1, 0.0))
    return sc, ph, seq


_REF = {}


def reference(key, n_coils, moving=False):
    import oracle
    k = (key, n_coils, moving)
    if k not in _REF:
        sc, ph, seq = coil_case(key, n_coils, moving)
        _REF[k] = oracle.simulate(sc, ph, seq, mode=oracle.MODE_BLOCK)
    return _REF[k]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("key,n_coils,moving", [("epi_small", 8, False), ("mrf40", 3, False),
                                                ("epi_small", 4, True), ("gre", 5, False)])
def test_coils_match_oracle(ctx, prec, key, n_coils, moving):
    sc, ph, seq = coil_case(key, n_coils, moving)
    ref = reference(key, n_coils, moving)
    ctx.set_config(prec)
    got = ctx.simulate(sc, ph, seq)
    assert got.shape == ref.shape == (n_coils, ph.n_groups, seq.n_adc)
    check(got, ref, prec, f"coils {key} x {n_coils}{' moving' if moving else ''}")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_unit_sensitivity_is_bitwise_the_plain_signal(ctx, prec):
    sc, ph, seq = case("epi_small")
    ctx.set_config(prec)
    a = ctx.simulate(sc, ph, seq)
    one = W.Phantom(ph.x, ph.y, ph.z, ph.pd, ph.t1, ph.t2, ph.dw, sens=np.ones((1, ph.n), np.complex64))
    b = ctx.simulate(sc, one, seq)
    assert b.shape == (1,) + a.shape and np.array_equal(a, b[0])


def test_coils_device_request_checkpoint_and_validation(ctx, K):
    import torch
    sc, ph, seq = coil_case("epi_small", 4)
    ctx.set_config("mixed")
    a = ctx.simulate(sc, ph, seq)
    dph = K.device_phantom(ph)
    sig = torch.zeros((4, ph.n_groups, seq.n_adc, 2), dtype=torch.float64, device="cuda:0")
    ctx.simulate(sc, dph, seq, where="device", sig=sig)
    b = sig.cpu().numpy()
    assert np.array_equal(a, b[..., 0] + 1j * b[..., 1])
    # chunked request with a checkpoint taken half way and restored into a fresh request
    req = ctx.open(sc, ph, seq, "host")
    req.advance(300)
    torch.cuda.synchronize()
    blob = req.save()
    req2 = ctx.open(sc, ph, seq, "host")
    req2.load(blob)
    while not req2.done():
        req2.advance(300)
    c = req2.result()
    req.close()
    req2.close()
    assert np.array_equal(a, c)
    bad = W.with_coils(case("epi_small")[1], 4)
    bad.sens = bad.sens.copy()
    bad.sens[2, 7] = np.nan
    with pytest.raises(K.KomaError) as e:
        ctx.simulate(sc, bad, seq)
    assert e.value.status == -2
    with pytest.raises(K.KomaError) as e:
        ctx.simulate(sc, K.device_phantom(bad), seq, where="device", sig=sig)
    assert e.value.status == -2


def test_coils_launch_shape_invariance(ctx):
    """Spins per lane and the partial budget (chunking over coils) do not
    change the mixed result beyond rounding; FP64 agrees to 1e-12."""
    sc, ph, seq = coil_case("epi_small", 8)
    ctx.set_config("fp64")
    base = ctx.simulate(sc, ph, seq)
    for kw in (dict(spins_per_lane=1), dict(spins_per_lane=4, partial_budget=1 << 20)):
        ctx.set_config("fp64", **kw)
        got = ctx.simulate(sc, ph, seq)
        assert worst(got, base) < 1e-12, kw
    ctx.set_config("fp64", spins_per_lane=0, partial_budget=1 << 30)
