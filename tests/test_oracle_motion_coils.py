"""Pins of the oracle's motion and receive-coil extensions.

Motion (section "Overview": a displacement field u(x, t) of the phantom;
experiment (d): u_y = v_y t): a spin sits at x + v t. The oracle takes the
field at the grid points with the position updated to each point and uses
the trapezoidal rule, as for static spins, so
  * on a gradient that is linear in time with the spin moving, the
    integrand G(t) . x(t) is quadratic and the rule's error over an interval
    of length h is the textbook (h^3 / 12) f''; it cancels over the two ramps
    of a symmetric trapezoid, so a bipolar velocity-encoding gradient gives
    the closed-form phase -gamma v M1 (M1 = first moment) on the minimal grid;
  * on an asymmetric lobe the oracle's phase equals the exact phase plus that
    error term, and the error falls as 1/m^2 when each ramp is cut into m
    pieces (the paper: with motion, intermediate points are needed).
Coils (section "Overview": coil sensitivities; section "Limitations"): coil
c's signal is the sum of sens_c * Mxy, checked against a superposition of
independent single-spin runs.
"""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W

GAMMA = W.GAMMA
SC = W.Scanner()


def f32(v):
    """The value the oracle reads (phantom arrays are float32)."""
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def spins(x, vx, pd=1.0):
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    vx = np.broadcast_to(np.asarray(vx, dtype=np.float64), x.shape)
    n = x.shape[0]
    z = np.zeros(n)
    inf = np.full(n, np.inf)
    return W.Phantom(x, z, z, np.full(n, pd), inf, inf, z, vx=vx, vy=z, vz=z)


def excite_then(lobes, adc_at_end=True):
    """Hard 90 deg about x (20 us, no gradient), then gradient lobes along x
    (list of (amp, rise, flat, fall)) back to back, then one ADC sample."""
    blocks = [W.Block(20e-6, rf=W.RFTrain(0.0, 20e-6, np.array([(np.pi / 2) / (GAMMA * 20e-6)])))]
    for amp, r, f, d in lobes:
        blocks.append(W.Block(r + f + d, gx=W.Trap(amp, 0.0, r, f, d)))
    blocks.append(W.Block(10e-6, adc=W.ADCWindow(10e-6, 0.0, 1)))
    return blocks


def to_seq(blocks, **caps):
    from oracle import discretize
    return W.make_sequence(*discretize.discretize(blocks, **caps))


def simpson_moments(lobes, t0):
    """Zeroth and first moments (T s/m, T s^2/m) of trapezoid lobes starting
    at t0, by Simpson's rule on each linear piece (exact for G and G t)."""
    m0 = m1 = 0.0
    t = t0
    for amp, r, f, d in lobes:
        for (ta, ga), (tb, gb) in (((t, 0.0), (t + r, amp)), ((t + r, amp), (t + r + f, amp)),
                                   ((t + r + f, amp), (t + r + f + d, 0.0))):
            tm, gm = 0.5 * (ta + tb), 0.5 * (ga + gb)
            h = tb - ta
            m0 += h / 6 * (ga + 4 * gm + gb)
            m1 += h / 6 * (ga * ta + 4 * gm * tm + gb * tb)
        t += r + f + d
    return m0, m1


@pytest.mark.parametrize("mode", [0, 1])
def test_zero_velocity_equals_static(oracle_mod, mode):
    sc, ph, seq = W.config(1)
    ph = ph.subset(np.arange(0, ph.n, 17))
    a = oracle_mod.simulate(sc, ph, seq, mode=mode)
    b = oracle_mod.simulate(sc, W.with_velocity(ph, (0.0, 0.0, 0.0)), seq, mode=mode)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("mode", [0, 1])
def test_velocity_encoding_bipolar_closed_form(oracle_mod, mode):
    """Bipolar symmetric trapezoids (areas +A, -A): static spins refocus
    wherever they are, moving spins gain -gamma v M1 with M1 = -A (2r + f)."""
    amp, r, f = 0.02, 200e-6, 1e-3
    seq = to_seq(excite_then([(amp, r, f, r), (-amp, r, f, r)]))
    xs = np.array([0.0, 0.03, -0.07, 0.0, 0.05, -0.02])
    vs = np.array([0.0, 0.0, 0.0, 0.1, -0.3, 0.7])
    s = oracle_mod.simulate(SC, spins(xs, vs), seq, mode=mode)[0, 0]
    one = oracle_mod.simulate(SC, spins([0.0], [0.0]), seq, mode=mode)[0, 0]
    m1 = -amp * (r + f) * (2 * r + f)
    want = one * np.sum(np.exp(-1j * GAMMA * f32(vs) * m1))
    assert abs(one - 1j) < 1e-12  # the 90 deg pulse about x puts M on +y
    assert abs(s - want) < 1e-12 * len(xs)


@pytest.mark.parametrize("mode", [0, 1])
def test_moving_spin_trapezoid_error_on_ramps(oracle_mod, mode):
    """Asymmetric lobe: the oracle's phase = exact phase (Simpson moments)
    plus the trapezoidal rule's h^3/12 f'' per ramp interval; cutting every
    interval into m pieces divides that term by m^2."""
    amp, r1, f, r2 = 0.03, 100e-6, 500e-6, 700e-6
    lobes = [(amp, r1, f, r2)]
    x0, v = 0.04, 0.5
    m0, m1 = simpson_moments(lobes, 20e-6)
    exact = -GAMMA * (f32(x0) * m0 + v * m1)
    # f(t) = -gamma G(t) x(t): f'' = -2 gamma G' v on a ramp of slope G'
    corr1 = -GAMMA * v * amp * (r1 ** 2 - r2 ** 2) / 6.0  # on the minimal grid
    for m in (1, 2, 4):
        # cap r1 / m: the ramps are cut into m and 7 m equal pieces
        caps = {} if m == 1 else {"dt_max": r1 / m * (1 + 1e-9)}
        seq = to_seq(excite_then(lobes), **caps)
        s = oracle_mod.simulate(SC, spins([x0], [v]), seq, mode=mode)[0, 0]
        one = oracle_mod.simulate(SC, spins([0.0], [0.0]), seq, mode=mode)[0, 0]
        got = np.angle(s / one)
        p1, p2 = (1, 1) if m == 1 else (m, int(round(m * r2 / r1)))
        want = exact - GAMMA * v * amp * (r1 ** 2 / p1 ** 2 - r2 ** 2 / p2 ** 2) / 6.0
        d = (got - want + np.pi) % (2 * np.pi) - np.pi
        assert abs(d) < 1e-10, (m, got, want)
    assert abs(corr1) > 1e-3  # the error term is far above rounding


def test_unit_sensitivity_is_the_plain_sum(oracle_mod):
    sc, ph, seq = W.config(1)
    ph = ph.subset(np.arange(0, ph.n, 29))
    a = oracle_mod.simulate(sc, ph, seq)
    ph.sens = np.ones((1, ph.n), dtype=np.complex64)
    b = oracle_mod.simulate(sc, ph, seq)
    assert b.shape == (1,) + a.shape
    assert np.array_equal(a, b[0])


def test_coil_signal_is_weighted_superposition(oracle_mod):
    """Coil c = sum_s sens_c(s) x (that spin's signal alone), groups kept."""
    rng = np.random.default_rng(11)
    seq = W.random_sequence(rng, 60, p_rf=0.3)
    ph = W.random_spins(rng, 7)
    ph.group_off = np.array([0, 3, 7])
    ph.sens = (rng.normal(size=(3, 7)) + 1j * rng.normal(size=(3, 7))).astype(np.complex64)
    got = oracle_mod.simulate(SC, ph, seq, mode=1)
    assert got.shape == (3, 2, seq.n_adc)
    want = np.zeros_like(got)
    for s in range(7):
        one = ph.subset([s])
        one.sens = None
        sig = oracle_mod.simulate(SC, one, seq, mode=1)[0]
        g = 0 if s < 3 else 1
        want[:, g, :] += ph.sens[:, s].astype(np.complex128)[:, None] * sig[None, :]
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_sensitivity_multiplies_mxy_unconjugated(oracle_mod):
    rng = np.random.default_rng(12)
    seq = W.random_sequence(rng, 40, p_rf=0.5)
    ph = W.random_spins(rng, 1)
    plain = oracle_mod.simulate(SC, ph, seq)[0]
    ph.sens = np.array([[1j, 2.0 + 0.5j]], dtype=np.complex64).T
    got = oracle_mod.simulate(SC, ph, seq)[:, 0, :]
    assert np.allclose(got[0], 1j * plain, rtol=0, atol=1e-15)
    assert np.allclose(got[1], (2.0 + 0.5j) * plain, rtol=1e-15, atol=1e-15)
