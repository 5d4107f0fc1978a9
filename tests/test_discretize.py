"""Sequence-aware time stepping (section "Simulation blocks, Regime
Switching, and Sequence-Aware Time Stepping").

Pins of the plain reference discretiser (``oracle/discretize.py``):
  * on sequences whose events all sit on a raster, the grid capped at the
    raster step is exactly the raster grid that ``workloads.UniformSeq``
    builds point by point (an independent construction);
  * closed-form point sets of hand-made blocks;
  * the minimal grid and the raster grid give the same FP64 signal, to the
    rounding of the accumulated phase (the paper's exactness claim for
    piecewise-linear G);
  * cutting RF samples finer (dt_rf_max) under a constant gradient leaves
    the FP64 signal unchanged (exactness for piecewise-constant B1), while
    under a ramp it moves it by the O(dt^3)-per-step splitting error.
Then the library's ``koma_discretize`` (host code of the C ABI) is checked
against the reference element by element, including its error codes.
"""
import ctypes
import math

import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W

GAMMA = W.GAMMA
SC = W.Scanner()


@pytest.fixture(scope="module")
def K():
    from paper_2301_02702_amd import build, komahip
    if build.stale():
        build.build()
    komahip.lib()
    return komahip


@pytest.fixture(scope="module")
def D():
    from oracle import discretize
    return discretize


def nrmse(a, b):
    return float(np.sqrt(np.mean(np.abs(a - b) ** 2)) / np.max(np.abs(b)))


def phase_scale(seq, ph):
    """Largest accumulated precession phase (rad) any spin can reach: the
    bound on the rounding of two FP64 phase sums over different grids."""
    dt = np.diff(seq.t)
    g = np.stack([seq.gx, seq.gy, seq.gz], 1)
    area = np.sum(0.5 * (np.abs(g[1:]) + np.abs(g[:-1])) * dt[:, None], 0)
    r = np.max(np.abs(np.stack([ph.x, ph.y, ph.z], 1)), 0)
    return GAMMA * float(np.dot(area, r)) + float(np.max(np.abs(ph.dw))) * float(seq.t[-1] - seq.t[0])


def check_same_grid(got, ref, g_rtol=1e-12):
    t, g, b1, adc = got
    assert len(t) == ref.n_t
    assert np.max(np.abs(t - ref.t)) <= 1e-15 * max(1.0, ref.t[-1]) * 8
    gref = np.stack([ref.gx, ref.gy, ref.gz], 1)
    assert np.max(np.abs(g - gref)) <= g_rtol * np.max(np.abs(gref))
    assert np.array_equal(b1, ref.b1)
    assert np.array_equal(adc, ref.adc_idx)


def as_tuple(seq):
    return seq.t, np.stack([seq.gx, seq.gy, seq.gz], 1), seq.b1, seq.adc_idx


# ------------------------------------------------------------ reference pins
@pytest.mark.parametrize("which", ["epi", "gre"])
def test_reference_reproduces_raster_builds(D, which):
    """Blocks capped at the raster step give the raster grid of the point-wise builder."""
    if which == "epi":
        blocks, ref, dt = W.epi_blocks(), W.epi_sequence(), 4e-6
    else:
        blocks, ref, dt = W.gre_blocks(n=16), W.gre_sequence(n=16), 10e-6
    check_same_grid(D.discretize(blocks, dt_max=dt), ref)


def test_reference_closed_form_points(D):
    """Hand-made blocks: the minimal grid is the union of block boundaries,
    trapezoid corners, waveform vertices, RF sample edges and ADC times."""
    ms = 1e-3
    blocks = [
        W.Block(1 * ms, rf=W.RFTrain(0.2 * ms, 0.1 * ms, np.array([1e-6, 2e-6, 3e-6]))),
        W.Block(2 * ms, gx=W.Trap(0.01, 0.25 * ms, 0.125 * ms, 0.5 * ms, 0.125 * ms),
                gy=W.PWL(np.array([0.0, 0.5 * ms]), np.array([0.0, 0.004])),
                adc=W.ADCWindow(0.375 * ms, 0.125 * ms, 5)),
        W.Block(0.5 * ms),
    ]
    t, g, b1, adc = D.discretize(blocks)
    want = [0, 0.2, 0.3, 0.4, 0.5, 1.0,             # RF edges, block edges
            1.0 + 0.25, 1.0 + 0.375, 1.0 + 0.875, 1.0 + 1.0,  # trapezoid corners
            1.0 + 0.5,                               # waveform vertices (0 and 0.5 ms)
            1.0 + 0.5, 1.0 + 0.625, 1.0 + 0.75,      # ADC samples 0.375 + k 0.125
            1.0 + 0.375, 1.0 + 0.875,
            3.0, 3.5]
    want = np.unique(np.array(want) * ms)
    assert len(t) == len(want) and np.max(np.abs(t - want)) < 1e-18
    assert np.array_equal(b1[:5], [0, 1e-6, 2e-6, 3e-6, 0]) and np.all(b1[5:] == 0)
    assert np.array_equal(t[adc], np.array([1.375, 1.5, 1.625, 1.75, 1.875]) * ms) or \
        np.max(np.abs(t[adc] - np.array([1.375, 1.5, 1.625, 1.75, 1.875]) * ms)) < 1e-18
    # trapezoid corners and waveform vertices hold their exact amplitudes
    def at(tm):
        return g[int(np.argmin(np.abs(t - tm * ms)))]
    # (to the rounding of the block-local time of each point)
    ap = lambda v: pytest.approx(v, rel=1e-12, abs=1e-18)  # noqa: E731
    assert at(1.25)[0] == ap(0.0) and at(1.375)[0] == ap(0.01) and at(1.875)[0] == ap(0.01)
    assert at(2.0)[0] == ap(0.0) and at(1.5)[1] == ap(0.004) and at(1.0)[1] == ap(0.0)
    assert at(1.625)[1] == 0.0
    # dt caps: RF samples cut in four, idle stretches cut to <= 0.3 ms
    t2, _, b2, _ = D.discretize(blocks, dt_max=0.3 * ms, dt_rf_max=0.025 * ms)
    rf_pts = np.sum((t2 >= 0.2 * ms - 1e-15) & (t2 <= 0.5 * ms + 1e-15))
    assert rf_pts == 13
    assert np.max(np.diff(t2)) <= 0.3 * ms * (1 + 1e-9)
    assert np.count_nonzero(b2) == 12


def test_minimal_grid_signal_equals_raster_grid(D, oracle_mod):
    """Only the vertices of G matter in precession: the minimal grid of the
    gradient echo (about 6x fewer intervals) gives the raster grid's signal."""
    sc, ph, ref = W.config(1)
    t, g, b1, adc = D.discretize(W.gre_blocks())
    m = W.make_sequence(t, g, b1, adc)
    assert m.n_int < ref.n_int / 5
    a = oracle_mod.simulate(sc, ph, ref, mode=oracle_mod.MODE_BLOCK)
    b = oracle_mod.simulate(sc, ph, m, mode=oracle_mod.MODE_BLOCK)
    tol = 64 * np.finfo(float).eps * phase_scale(ref, ph)
    err = nrmse(b, a)
    assert err < tol, (err, tol)
    # the same in per-interval splitting mode, on the EPI
    sc, ph, ref = W.config(2)
    ph = ph.subset(np.arange(0, ph.n, 97))
    t, g, b1, adc = D.discretize(W.epi_blocks())
    m = W.make_sequence(t, g, b1, adc)
    a = oracle_mod.simulate(sc, ph, ref, mode=oracle_mod.MODE_STEP)
    b = oracle_mod.simulate(sc, ph, m, mode=oracle_mod.MODE_STEP)
    assert nrmse(b, a) < 64 * np.finfo(float).eps * phase_scale(ref, ph)


def _slice_blocks(ramp_under_rf: bool):
    """A sinc RF train played on a flat gradient, or over a ramp, then an ADC."""
    ms = 1e-3
    rf = W.sinc_pulse(40, 20e-6, np.pi / 3, 2.0)
    if ramp_under_rf:
        gz = W.Trap(0.02, 0.0, 0.8 * ms, 0.0, 0.2 * ms)  # RF rides the up-ramp
    else:
        gz = W.Trap(0.02, 0.0, 0.05 * ms, 0.9 * ms, 0.05 * ms)
    return [W.Block(1.0 * ms, gz=gz, rf=W.RFTrain(0.1 * ms, 20e-6, rf)),
            W.Block(0.5 * ms, gz=W.Trap(-0.02, 0.0, 0.05 * ms, 0.4 * ms, 0.05 * ms)),
            W.Block(0.2 * ms, adc=W.ADCWindow(0.1 * ms, 10e-6, 3))]


def test_rf_subdivision_exact_for_piecewise_constant_b1(D, oracle_mod):
    """Eq. Rot_exc solves the rotation part of the Bloch equation exactly
    for a constant field: without relaxation (which the splitting applies
    after each rotation), cutting each RF sample in 4 under a flat gradient
    leaves the signal unchanged; over a ramp the field varies inside a
    sample and the cut moves the result."""
    rng = np.random.default_rng(5)
    ph = W.random_spins(rng, 300, extent=0.01, dw_max=300.0)
    ph.t1 = np.full(ph.n, np.inf, dtype=np.float32)
    ph.t2 = np.full(ph.n, np.inf, dtype=np.float32)
    out = {}
    for ramp in (False, True):
        blocks = _slice_blocks(ramp)
        s1 = W.make_sequence(*D.discretize(blocks))
        s4 = W.make_sequence(*D.discretize(blocks, dt_rf_max=5e-6))
        assert s1.n_rf == 40 and s4.n_rf == 160
        a = oracle_mod.simulate(SC, ph, s1, mode=oracle_mod.MODE_STEP)
        b = oracle_mod.simulate(SC, ph, s4, mode=oracle_mod.MODE_STEP)
        out[ramp] = nrmse(b, a)
    assert out[False] < 1e-12, out
    assert out[True] > 1e-7, out


# ------------------------------------------------------------ library vs reference
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("caps", [(math.inf, math.inf), (50e-6, 3e-6)])
def test_library_matches_reference_on_random_blocks(K, D, seed, caps):
    blocks = W.random_blocks(np.random.default_rng(seed), 40)
    got = K.koma_discretize(blocks, *caps)
    t, g, b1, adc = D.discretize(blocks, *caps)
    assert got.n_t == len(t) and got.n_adc == len(adc)
    assert np.max(np.abs(got.t - t)) <= 1e-15
    gg = np.stack([got.gx, got.gy, got.gz], 1)
    assert np.max(np.abs(gg - g)) <= 1e-12 * max(np.max(np.abs(g)), 1e-30)
    assert np.array_equal(got.b1, b1)
    assert np.array_equal(got.adc_idx, adc)
    if not math.isinf(caps[0]):
        rf = got.b1 != 0
        d = np.diff(got.t)
        assert np.all(d[~rf] <= caps[0] * (1 + 1e-9)) and np.all(d[rf] <= caps[1] * (1 + 1e-9))


@pytest.mark.parametrize("which", ["epi", "gre"])
def test_library_reproduces_raster_builds(K, which):
    if which == "epi":
        blocks, ref, dt = W.epi_blocks(), W.epi_sequence(), 4e-6
    else:
        blocks, ref, dt = W.gre_blocks(), W.gre_sequence(), 10e-6
    check_same_grid(as_tuple(K.koma_discretize(blocks, dt_max=dt)), ref)
    m = K.koma_discretize(blocks)
    assert m.n_adc == ref.n_adc and m.n_int < ref.n_int


def test_library_minimal_grid_feeds_the_planner(K):
    """The discretised sequence is a valid simulator input."""
    m = K.koma_discretize(W.epi_blocks())
    info = K.koma_plan_info(SC, W.single_spin(), m, K.make_config())
    assert info["n_adc"] == 16384 and info["n_rf"] == 50


def _bad(K, blocks, dt_max=math.inf, dt_rf_max=math.inf):
    with pytest.raises(K.KomaError) as e:
        K.koma_discretize(blocks, dt_max, dt_rf_max)
    assert "koma_discretize" in str(e.value)
    return e.value.status


def test_library_rejects_bad_blocks(K):
    ms = 1e-3
    ok = W.Block(1 * ms, gx=W.Trap(0.01, 0, 0.1 * ms, 0.2 * ms, 0.1 * ms))
    assert K.koma_discretize([ok]).n_t == 5
    assert _bad(K, [W.Block(0.0)]) == -3
    assert _bad(K, [W.Block(0.3 * ms, gx=W.Trap(0.01, 0, 0.1 * ms, 0.2 * ms, 0.1 * ms))]) == -3  # past end
    assert _bad(K, [W.Block(1 * ms, gx=W.Trap(0.01, 0, 0.0, 0.2 * ms, 0.1 * ms))]) == -3  # rise 0
    assert _bad(K, [W.Block(1 * ms, gy=W.PWL(np.array([0.0, 0.0]), np.array([0.0, 0.0])))]) == -3
    assert _bad(K, [W.Block(1 * ms, gy=W.PWL(np.array([0.1, 0.2]) * ms, np.array([0.01, 0.0])))]) == -3
    # a waveform ending at the block end must meet the next block's value
    a = W.Block(1 * ms, gy=W.PWL(np.array([0.5, 1.0]) * ms, np.array([0.0, 0.01])))
    b = W.Block(1 * ms, gy=W.PWL(np.array([0.0, 0.5]) * ms, np.array([0.01, 0.0])))
    assert K.koma_discretize([a, b]).n_t == 5
    assert _bad(K, [a, ok]) == -3
    assert _bad(K, [W.Block(1 * ms, rf=W.RFTrain(0.5 * ms, 0.1 * ms, np.ones(6) * 1e-6))]) == -3
    assert _bad(K, [W.Block(1 * ms, rf=W.RFTrain(0.0, 0.1 * ms, np.array([np.nan])))]) == -3
    assert _bad(K, [W.Block(1 * ms, adc=W.ADCWindow(0.0, 0.2 * ms, 7))]) == -3
    two = [W.Block(1 * ms, adc=W.ADCWindow(1 * ms, 0.0, 1)), W.Block(1 * ms, adc=W.ADCWindow(0.0, 0.0, 1))]
    assert _bad(K, two) == -3  # two samples at one instant
    assert _bad(K, [ok], dt_max=0.0) == -1
    assert _bad(K, [ok], dt_rf_max=-1.0) == -1
    assert _bad(K, []) == -1


def test_library_two_call_protocol(K):
    """Size query, then a call with capacities; short capacities are rejected."""
    blocks = W.random_blocks(np.random.default_rng(9), 10)
    b = K._BlockArgs(blocks)
    L = K.lib()
    n_t, n_adc = ctypes.c_int64(0), ctypes.c_int64(0)
    assert L.koma_discretize(b.c, b.n, math.inf, math.inf, ctypes.byref(n_t), ctypes.byref(n_adc),
                             *([None] * 7)) == 0
    nt, na = n_t.value, n_adc.value
    bufs = [np.zeros(nt) for _ in range(4)] + [np.zeros(nt - 1) for _ in range(2)]
    adc = np.zeros(max(na, 1), dtype=np.int64)
    ptrs = [x.ctypes.data for x in bufs] + [adc.ctypes.data]
    n_t.value = nt - 1
    assert L.koma_discretize(b.c, b.n, math.inf, math.inf, ctypes.byref(n_t), ctypes.byref(n_adc), *ptrs) == -1
    n_t.value = nt
    assert L.koma_discretize(b.c, b.n, math.inf, math.inf, ctypes.byref(n_t), ctypes.byref(n_adc), *ptrs) == 0
    assert n_t.value == nt and n_adc.value == na
    # an unknown gradient kind is an argument error
    b.c[0].g[0].kind = 7
    assert L.koma_discretize(b.c, b.n, math.inf, math.inf, ctypes.byref(n_t), ctypes.byref(n_adc),
                             *([None] * 7)) == -1
