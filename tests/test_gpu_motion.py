"""GPU parity of moving spins (x(t) = x + v t) against the FP64 oracle.

The paper's motion example (experiment (d)): the EPI of (c) with the
phantom moving along y at v_y = 0.1 m/s. Here the head-like phantom of the
EPI tests takes its place, at a size the oracle finishes in seconds.
Parity bar as in the static parity tests (tests/_gpu.py): NRMSE and the
largest sample error <= 1e-10 (FP64) and 1e-4 (mixed) of max|oracle|.
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


@pytest.fixture(scope="module")
def epi_moving():
    import oracle
    sc, ph, seq = case("epi_small")
    mv = W.with_velocity(ph, (0.0, 0.1, 0.0))
    return sc, mv, seq, oracle.simulate(sc, mv, seq, mode=oracle.MODE_BLOCK)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_moving_epi_matches_oracle(ctx, epi_moving, prec):
    sc, ph, seq, ref = epi_moving
    say(f"[motion] epi_small v_y = 0.1 m/s {prec}")
    # every sample on its own (spin-sequential), then the lines as stretches
    # with the quadratic first-moment model (sample-parallel)
    ctx.set_config(prec, defer_min_adc=-1)
    check(ctx.simulate(sc, ph, seq), ref, prec, "motion epi_small, samples one by one")
    ctx.set_config(prec)
    got = ctx.simulate(sc, ph, seq)
    check(got, ref, prec, "motion epi_small, stretches")
    # the motion is visible: the static result differs from the moving one
    static = ctx.simulate(sc, W.Phantom(ph.x, ph.y, ph.z, ph.pd, ph.t1, ph.t2, ph.dw), seq)
    d = float(np.max(nrmse(static, ref)))
    say(f"[motion] epi_small {prec}: static differs by {d:.3e}")
    assert d > 100 * TOL["mixed"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_moving_random_sequences(ctx, prec, seed):
    """Random grids (random piecewise-linear G, complex B1 on half of the
    intervals, random ADC points) with spins of random velocities; ragged
    spin counts over several tiles."""
    import oracle
    rng = np.random.default_rng(900 + seed)
    seq = W.random_sequence(rng, 300, p_rf=0.4, g_max=0.02)
    ph = W.random_spins(rng, 130 + 61 * seed, extent=0.05, dw_max=300.0)
    ph = W.with_velocity(ph, rng.uniform(-0.5, 0.5, 3), spread=0.3, seed=seed)
    ref = oracle.simulate(W.Scanner(), ph, seq, mode=oracle.MODE_STEP)
    for dm, spl in ((32, 0), (-1, 0), (0, 1), (2, 8)):  # inline samples and stretches of every length
        ctx.set_config(prec, defer_min_adc=dm, spins_per_lane=spl)
        got = ctx.simulate(W.Scanner(), ph, seq)
        check(got, ref, prec, f"motion random seed {seed} defer {dm}: {ph.n} spins")
    ctx.set_config(prec, defer_min_adc=32, spins_per_lane=0)


def test_velocity_encoding_phase_on_gpu(ctx, K):
    """Bipolar symmetric trapezoids: the phase of a moving spin is
    -gamma v M1 (closed form), static spins refocus."""
    amp, r, f = 0.02, 200e-6, 1e-3
    blocks = [W.Block(20e-6, rf=W.RFTrain(0.0, 20e-6, np.array([(np.pi / 2) / (W.GAMMA * 20e-6)]))),
              W.Block(2 * r + f, gx=W.Trap(amp, 0.0, r, f, r)),
              W.Block(2 * r + f, gx=W.Trap(-amp, 0.0, r, f, r)),
              W.Block(10e-6, adc=W.ADCWindow(10e-6, 0.0, 1))]
    seq = K.koma_discretize(blocks)
    vs = np.array([0.0, 0.1, -0.3, 0.7, 0.05], dtype=np.float32).astype(np.float64)
    xs = np.array([0.0, 0.02, -0.04, 0.01, 0.0])
    m1 = -amp * (r + f) * (2 * r + f)
    for prec, tol in (("fp64", 1e-12), ("mixed", 5e-6)):
        ctx.set_config(prec)
        for x, v in zip(xs, vs):
            z = np.zeros(1)
            ph = W.Phantom([x], z, z, [1.0], [np.inf], [np.inf], z, vx=[v], vy=z, vz=z)
            s = ctx.simulate(W.Scanner(), ph, seq)[0, 0]
            want = 1j * np.exp(-1j * W.GAMMA * v * m1)
            assert abs(s - want) < tol, (prec, x, v, s, want)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_zero_velocity_matches_static_path(ctx, prec):
    sc, ph, seq = case("gre")
    ctx.set_config(prec)
    a = ctx.simulate(sc, ph, seq)
    b = ctx.simulate(sc, W.with_velocity(ph, (0.0, 0.0, 0.0)), seq)
    e = float(np.max(nrmse(b, a)))
    say(f"[motion] v = 0 vs static path {prec}: {e:.3e}")
    assert e <= (1e-12 if prec == "fp64" else 2e-6)


def test_moving_device_phantom_and_request_path(ctx, K, epi_moving):
    """Device-resident moving phantom and the chunked request path give the
    host-phantom result bitwise; a non-finite velocity is rejected."""
    import torch
    sc, ph, seq, _ = epi_moving
    ctx.set_config("mixed")
    a = ctx.simulate(sc, ph, seq)
    dph = K.device_phantom(ph)
    sig = torch.zeros((ph.n_groups, seq.n_adc, 2), dtype=torch.float64, device="cuda:0")
    ctx.simulate(sc, dph, seq, where="device", sig=sig)
    b = sig.cpu().numpy()
    assert np.array_equal(a, b[..., 0] + 1j * b[..., 1])
    req = ctx.open(sc, ph, seq, "host")
    while not req.done():
        req.advance(700)
    c = req.result()
    req.close()
    assert np.array_equal(a, c)
    bad = W.with_velocity(ph)
    bad.vz = bad.vz.copy()
    bad.vz[5] = np.inf
    with pytest.raises(K.KomaError) as e:
        ctx.simulate(sc, bad, seq)
    assert e.value.status == -2
    dbad = K.device_phantom(bad)
    with pytest.raises(K.KomaError) as e:
        ctx.simulate(sc, dbad, seq, where="device", sig=sig)
    assert e.value.status == -2
