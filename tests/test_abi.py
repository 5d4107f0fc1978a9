"""C-ABI contract on the host: the library loads, exports every entry point
the header declares, plans sequences on the host and rejects bad inputs with
the documented status codes. No device work is done here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def K():
    from paper_2301_02702_amd import build, komahip
    if build.stale():
        build.build()
    komahip.lib()
    return komahip


def header_functions():
    src = open(os.path.join(ROOT, "include", "komahip.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(koma_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(K):
    names = header_functions()
    assert len(names) >= 18
    L = ctypes.CDLL(K.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(K.EXPORTS), set(names) ^ set(K.EXPORTS)


def test_config_defaults(K):
    c = K.make_config()
    assert c.precision == K.KOMA_MIXED and c.wg_size == 256 and c.spins_per_lane == 0
    assert c.defer_min_adc == 32 and c.stretch_max == 128 and c.partial_budget == 1 << 30
    assert c.tile_packing == 1


@pytest.mark.parametrize("k,expect", [
    # one readout gradient for every GRE line; two readout polarities in EPI
    # identical consecutive excitation intervals are one event: the two
    # middle samples of each GRE sinc, the EPI hard pulse, each MRF hard pulse
    (1, dict(n_rf=6400, n_rf_events=6336, n_runs=64, n_deferred_adc=4096, n_inline_adc=0, n_stretches=64,
             n_families=1, n_snapshots=64)),
    (2, dict(n_rf=50, n_rf_events=1, n_runs=1, n_deferred_adc=16384, n_inline_adc=0, n_stretches=128,
             n_families=2, n_snapshots=1)),
    (4, dict(n_rf=10000, n_rf_events=1000, n_runs=1000, n_deferred_adc=0, n_inline_adc=1000, n_stretches=0,
             n_families=0, n_snapshots=0)),
])
def test_host_plans_of_the_workloads(K, k, expect):
    sc, ph, seq = W.config(k)
    info = K.koma_plan_info(sc, ph, seq, K.make_config(tile_packing=0))
    for key, v in expect.items():
        assert info[key] == v, (key, info[key], v)
    assert info["n_tiles"] == sum(-(-int(b - a) // 64) for a, b in zip(
        *(lambda o: (o[:-1], o[1:]))(ph.group_off if ph.group_off is not None else np.array([0, ph.n]))))
    # one event per excitation interval, block end, snapshot and inline stretch
    assert info["n_events"] >= expect["n_rf_events"] + expect["n_runs"] + expect["n_snapshots"]


def test_stretches_split_at_the_length_cap(K):
    sc, ph, seq = W.config(2)
    for smax, want, fams in ((128, 128, 2), (100, 256, 2), (1, 16384, 1)):
        info = K.koma_plan_info(sc, ph, seq, K.make_config(stretch_max=smax))
        assert info["n_stretches"] == want
        # single samples have no increments: one family takes them all
        assert info["n_families"] == fams


def test_runs_of_identical_excitation_intervals_are_one_event(K):
    """Equal field values and lengths equal up to the rounding of the time
    grid merge; a changed field, a sample or a precession interval in between
    ends the run."""
    ph = W.random_spins(np.random.default_rng(4), 10)
    dt = 4e-6
    b1 = np.full(40, 1e-5 + 0j)
    b1[17] = 1.1e-5          # one different value: runs 17, 1, 22
    seq = W.make_sequence(dt * np.arange(41), np.zeros((41, 3)), b1, [])
    info = K.koma_plan_info(W.Scanner(), ph, seq, K.make_config())
    assert info["n_rf"] == 40 and info["n_rf_events"] == 3
    seq = W.make_sequence(dt * np.arange(41), np.zeros((41, 3)), np.full(40, 1e-5 + 0j), [10, 30])
    info = K.koma_plan_info(W.Scanner(), ph, seq, K.make_config())
    assert info["n_rf_events"] == 3       # split at the two sampled points
    g = np.zeros((41, 3))
    g[20:, 0] = 1e-3                       # the field changes at point 20 (mean G of interval 19)
    seq = W.make_sequence(dt * np.arange(41), g, np.full(40, 1e-5 + 0j), [])
    info = K.koma_plan_info(W.Scanner(), ph, seq, K.make_config())
    assert info["n_rf_events"] == 3       # runs 0..18, 19, 20..39
    t = dt * np.arange(41)
    t[25:] += 1e-9                         # one longer interval
    seq = W.make_sequence(t, np.zeros((41, 3)), np.full(40, 1e-5 + 0j), [])
    info = K.koma_plan_info(W.Scanner(), ph, seq, K.make_config())
    assert info["n_rf_events"] == 3


def test_runs_of_single_intervals_for_the_one_lane_kernel(K):
    """Consecutive single excitation intervals (distinct fields, as in a
    shaped pulse under a slice-select gradient) whose relaxation keys are
    equal form one run of the one-lane kernel: the run ends where the
    interval length changes by more than the time grid's rounding, and a run
    of identical intervals (one event with a count) or a sample in between
    ends it too."""
    ph = W.random_spins(np.random.default_rng(5), 10)
    dt = 4e-6
    b1 = (1e-5 * np.sinc(np.linspace(-3, 3, 100)) + 0j) * np.exp(0.3j * np.arange(100))
    t = dt * np.arange(101)
    g = np.zeros((101, 3))
    g[:, 2] = 10e-3                        # slice select
    info = K.koma_plan_info(W.Scanner(), ph, W.make_sequence(t, g, b1, []), K.make_config())
    assert info["n_rf_events"] == 100 and info["max_single_run"] == 100
    t2 = t.copy()
    t2[60:] += 1e-9                        # interval 59 longer: runs 0..58, 59, 60..99
    info = K.koma_plan_info(W.Scanner(), ph, W.make_sequence(t2, g, b1, []), K.make_config())
    assert info["max_single_run"] == 59
    b1r = b1.copy()
    b1r[30:40] = b1r[30]                   # ten identical intervals: one event with a count
    info = K.koma_plan_info(W.Scanner(), ph, W.make_sequence(t, g, b1r, []), K.make_config())
    assert info["n_rf_events"] == 91 and info["max_single_run"] == 60
    info = K.koma_plan_info(W.Scanner(), ph, W.make_sequence(t, g, b1, [45]), K.make_config())
    assert info["max_single_run"] == 55


def test_matrix_core_grid_fills_whole_rounds(K):
    """The matrix-core sample-parallel grids are sized to whole rounds of
    resident workgroups (256 CUs when there is no device). In the mixed form
    (3 per CU) a workgroup takes 4 or 6 stretches, whichever gives fewer
    rounds x tiles per wavefront x stretches (6 counted 3.5 % cheaper):
    epi256 keeps 4, with 11 tiles per wavefront, 24 spin blocks x 32 batches =
    768 workgroups (6 would need 8 tiles, 32 x 22 = 704 in the one round);
    a 1e6-spin GRE request takes 6 with 4 tiles, 977 blocks x 11 batches in
    14 rounds (4 would take 2 tiles, 1,954 x 16 in 41); a 1e5-spin one keeps
    4 (9 tiles, 44 blocks), since 6 would take more blocks (66) and so more
    partial sums. A grid of 32 or more rounds at 16 tiles per wavefront is
    searched on up to 32 tiles (SE-EPI).
    In FP64 (2 per CU, 64 KB of LDS each) every S fills whole rounds and the
    largest, 16, gives 16 blocks x 32 = 512 (one round); the vector-ALU forms
    keep 1, 2, 4 or 8. A requested batch size is kept, other values than 0,
    4 and 6 are rejected."""
    sc, ph, seq = W.config(2)
    i = K.koma_plan_info(sc, ph, seq, K.make_config())
    assert (i["spins_per_lane"], i["n_blocks"], i["stretches_per_wg"]) == (11, 24, 4)
    i = K.koma_plan_info(sc, ph, seq, K.make_config("fp64"))
    assert (i["spins_per_lane"], i["n_blocks"], i["stretches_per_wg"]) == (16, 16, 4)
    for n, want in ((1000000, (4, 977, 6, 64)), (100000, (9, 44, 4, 64))):
        r = W.ServingRequest(0, 0.0, n, "gre", 77)
        i = K.koma_plan_info(W.Scanner(), W.serving_phantom(r), W.serving_sequence("gre"), K.make_config())
        assert (i["spins_per_lane"], i["n_blocks"], i["stretches_per_wg"], i["n_stretches"]) == want, n
    # SE-EPI (1,221 blocks x 72 batches at S = 16: 115 rounds) goes on to
    # S = 32: 611 blocks x 72 batches, whole rounds to 0.5 %
    sc5, ph5, seq5 = W.config(5)
    i = K.koma_plan_info(sc5, ph5, seq5, K.make_config())
    assert (i["spins_per_lane"], i["n_blocks"], i["stretches_per_wg"]) == (32, 611, 6)
    i = K.koma_plan_info(sc5, ph5, seq5, K.make_config("fp64"))
    assert (i["spins_per_lane"], i["n_blocks"], i["stretches_per_wg"]) == (32, 611, 4)
    # a requested S keeps the smaller batch; a requested batch is kept
    i = K.koma_plan_info(sc, ph, seq, K.make_config(spins_per_lane=3))
    assert (i["spins_per_lane"], i["stretches_per_wg"]) == (3, 4)
    i = K.koma_plan_info(sc, ph, seq, K.make_config(stretches_per_wg=6))
    assert (i["spins_per_lane"], i["n_blocks"], i["stretches_per_wg"]) == (8, 32, 6)
    i = K.koma_plan_info(sc, ph, seq, K.make_config("fp64", stretches_per_wg=6))
    assert i["stretches_per_wg"] == 4
    for bad in (-1, 1, 5, 8):
        with pytest.raises(K.KomaError) as e:
            K.koma_plan_info(sc, ph, seq, K.make_config(stretches_per_wg=bad))
        assert e.value.status == -1
    for cfg in (K.make_config("fp64", sample_engine=1), K.make_config(sample_engine=1)):
        assert K.koma_plan_info(sc, ph, seq, cfg)["spins_per_lane"] in (1, 2, 4, 8)
    assert K.koma_plan_info(sc, W.with_velocity(ph.subset(np.arange(0, ph.n, 8))), seq,
                            K.make_config())["spins_per_lane"] in (1, 2, 4, 8)


def test_stretches_of_equal_increments_form_families(K):
    """Lines of equal readout amplitude share their per-sample increments
    (one family each); single samples join any family."""
    rng = np.random.default_rng(3)
    ph = W.random_spins(rng, 100)
    seq = W.readout_lines_sequence([0.01, -0.01, 0.01, 0.02, -0.01, 0.01, -0.01])
    info = K.koma_plan_info(W.Scanner(), ph, seq, K.make_config())
    assert info["n_stretches"] == 7 and info["n_families"] == 3
    info = K.koma_plan_info(W.Scanner(), ph, seq, K.make_config(stretch_max=16))
    assert info["n_stretches"] == 7 * 3 and info["n_families"] == 3
    info = K.koma_plan_info(W.Scanner(), ph, seq, K.make_config(stretch_max=1))
    assert info["n_families"] == 1


def test_defer_threshold_moves_samples_inline(K):
    sc, ph, seq = W.config(1)
    info = K.koma_plan_info(sc, ph, seq, K.make_config(defer_min_adc=-1))
    assert info["n_deferred_adc"] == 0 and info["n_inline_adc"] == 4096 and info["n_snapshots"] == 0
    info = K.koma_plan_info(sc, ph, seq, K.make_config(defer_min_adc=65))
    assert info["n_deferred_adc"] == 0


def _seq(**kw):
    t = np.array([0.0, 1e-3, 2e-3, 3e-3])
    d = dict(t=t, g=np.zeros((4, 3)), b1=np.array([1e-6, 0, 0], dtype=complex), adc=[1, 3])
    d.update(kw)
    return W.make_sequence(d["t"], d["g"], d["b1"], d["adc"])


@pytest.mark.parametrize("bad,code", [
    (dict(t=np.array([0.0, 1e-3, 1e-3, 3e-3])), -3),        # not strictly increasing
    (dict(t=np.array([0.0, np.nan, 2e-3, 3e-3])), -3),      # NaN time
    (dict(adc=[3, 1]), -3),                                 # ADC not increasing
    (dict(adc=[0, 4]), -3),                                 # ADC out of range
    (dict(b1=np.array([np.inf, 0, 0], dtype=complex)), -3),  # non-finite B1
])
def test_sequence_validation(K, bad, code):
    seq = _seq(**bad)
    with pytest.raises(K.KomaError) as e:
        K.koma_plan_info(W.Scanner(), W.single_spin(), seq, K.make_config())
    assert e.value.status == code


def test_phantom_and_config_validation(K):
    seq = _seq()
    ph = W.random_spins(np.random.default_rng(0), 10)
    ph.group_off = np.array([0, 5, 4, 10])
    with pytest.raises(K.KomaError) as e:
        K.koma_plan_info(W.Scanner(), ph, seq, K.make_config())
    assert e.value.status == -2
    ph.group_off = np.array([0, 5, 9])  # does not end at n
    with pytest.raises(K.KomaError) as e:
        K.koma_plan_info(W.Scanner(), ph, seq, K.make_config())
    assert e.value.status == -2
    ph.group_off = None
    for bad in (dict(spins_per_lane=17), dict(spins_per_lane=-1), dict(wg_size=128), dict(stretch_max=0), dict(stretch_max=129),
                dict(chunk_events=0), dict(partial_budget=1000)):
        with pytest.raises(K.KomaError) as e:
            K.koma_plan_info(W.Scanner(), ph, seq, K.make_config(**bad))
        assert e.value.status == -1, bad
    with pytest.raises(K.KomaError) as e:
        K.koma_plan_info(W.Scanner(gamma=-1.0), ph, seq, K.make_config())
    assert e.value.status == -1


def test_footprint_counts_snapshots_and_partials(K):
    sc, ph, seq = W.config(2)
    # the same launch shape in both forms (the planner's choices differ)
    f_mixed = K.koma_footprint(ph, seq, K.make_config("mixed", spins_per_lane=8))
    f_fp64 = K.koma_footprint(ph, seq, K.make_config("fp64", spins_per_lane=8))
    n_pad = 1024 * 64
    assert f_fp64 > f_mixed > n_pad * (8 + 12)  # snapshot + state at least


def test_moving_phantom_plans(K):
    """Moving spins: each EPI line is one stretch (moments linear, first
    moments quadratic in the sample index on the flat top); with deferral
    off, one event per sample."""
    sc, ph, seq = W.config(2)
    ph = ph.subset(np.arange(0, ph.n, 64))
    info = K.koma_plan_info(sc, W.with_velocity(ph), seq, K.make_config())
    assert info["n_deferred_adc"] == seq.n_adc and info["n_stretches"] == 128 and info["n_snapshots"] == 1
    info = K.koma_plan_info(sc, W.with_velocity(ph), seq, K.make_config(defer_min_adc=-1))
    assert info["n_deferred_adc"] == 0 and info["n_stretches"] == 0 and info["n_snapshots"] == 0
    assert info["n_inline_adc"] == seq.n_adc
    # one event per sample, per excitation run and per block end
    assert info["n_events"] == seq.n_adc + info["n_rf_events"] + info["n_runs"]
    f_static = K.koma_footprint(ph, seq, K.make_config())
    f_moving = K.koma_footprint(W.with_velocity(ph), seq, K.make_config())
    assert f_moving > f_static


def test_velocity_validation(K):
    seq = _seq()
    ph = W.random_spins(np.random.default_rng(0), 10)
    assert K.koma_plan_info(W.Scanner(), W.with_velocity(ph), seq, K.make_config())["n_spins"] == 10
    # a partial velocity set is an argument error
    p = K._PhantomArgs(W.with_velocity(ph), False)
    p.c.vy = None
    info = K.koma_req_info()
    sc = K.make_scanner(W.Scanner())
    s = K._SeqArgs(seq)
    cfg = K.make_config()
    st = K.lib().koma_plan_info(ctypes.byref(sc), ctypes.byref(p.c), ctypes.byref(s.c), ctypes.byref(cfg),
                                ctypes.byref(info))
    assert st == -1


def test_coil_plans_and_validation(K):
    sc, ph, seq = W.config(2)
    ph = ph.subset(np.arange(0, ph.n, 16))
    f1 = K.koma_footprint(ph, seq, K.make_config())
    pc = W.with_coils(ph, 8)
    f8 = K.koma_footprint(pc, seq, K.make_config())
    assert f8 > f1 + 8 * ph.n * 8  # sensitivities at least
    # (the same spin blocks in both: the planner's own choice also weighs the coils)
    i1 = K.koma_plan_info(sc, ph, seq, K.make_config(partial_budget=1 << 20, spins_per_lane=2))
    i8 = K.koma_plan_info(sc, pc, seq, K.make_config(partial_budget=1 << 20, spins_per_lane=2))
    assert i1["n_blocks"] == i8["n_blocks"]
    assert i8["n_chunks"] >= 4 * i1["n_chunks"]  # the partial budget is shared by the coils
    p = K._PhantomArgs(pc, False)
    info = K.koma_req_info()
    s = K._SeqArgs(seq)
    cfg = K.make_config()
    scc = K.make_scanner(sc)
    for mutate in (lambda c: setattr(c, "n_coils", 1025), lambda c: setattr(c, "sens_im", None),
                   lambda c: setattr(c, "n_coils", -1)):
        q = K._PhantomArgs(pc, False)
        mutate(q.c)
        st = K.lib().koma_plan_info(ctypes.byref(scc), ctypes.byref(q.c), ctypes.byref(s.c), ctypes.byref(cfg),
                                    ctypes.byref(info))
        assert st == -1
    assert p.n_coils == 8


def _plan_tiles(K, ph, seq, **cfg):
    i = K.koma_plan_info(W.Scanner(), ph, seq, K.make_config(**cfg))
    return i["n_tiles"], i["n_rows"]


def test_packed_tiles_cross_group_boundaries(K):
    """Without deferred samples and with every non-empty group >= 64 spins,
    wavefronts take 64 consecutive spins across groups: ceil(n / 64) tiles,
    one more partial row for every tile a group boundary cuts."""
    sc, ph, seq = W.config(4)  # 10,000 groups of 400 spins, one inline sample per TR
    assert _plan_tiles(K, ph, seq, tile_packing=0) == (70000, 70000)
    # boundaries at 400 g: inside a tile unless 400 g is a multiple of 64 (g % 4 == 0)
    assert _plan_tiles(K, ph, seq) == (62500, 62500 + 7500)
    rng = np.random.default_rng(5)
    sizes = rng.integers(64, 300, 40)
    sizes[[3, 17, 18]] = 0  # empty groups
    off = np.concatenate([[0], np.cumsum(sizes)])
    n = int(off[-1])
    sp = W.random_spins(rng, n)
    sp.group_off = off
    rseq = W.random_sequence(rng, 60, p_rf=0.3, p_adc=0.5)
    cuts = sum(1 for b in off[1:-1] if b % 64 != 0 and b < n)
    cut_tiles = len({int(b) // 64 for b in off[1:-1] if b % 64 != 0})
    assert cuts >= cut_tiles > 0
    assert _plan_tiles(K, sp, rseq, defer_min_adc=-1) == (-(-n // 64), -(-n // 64) + cut_tiles)
    # a group below 64 spins, or deferred samples: per-group tiles
    sizes2 = sizes.copy()
    sizes2[5] = 10
    sp.group_off = np.concatenate([[0], np.cumsum(sizes2)])
    sp2 = W.random_spins(rng, int(sp.group_off[-1]))
    sp2.group_off = sp.group_off
    per_group = sum(-(-int(z) // 64) for z in sizes2)
    assert _plan_tiles(K, sp2, rseq, defer_min_adc=-1) == (per_group, per_group)
    _, eph, eseq = W.config(2)
    eph.group_off = np.array([0, 30000, eph.n])
    t, r = _plan_tiles(K, eph, eseq)
    assert t == r == -(-30000 // 64) + -(-(eph.n - 30000) // 64)


def test_lanes_per_spin_of_the_planner(K):
    """Several lanes per spin while the tiles fill few wavefronts: the GRE
    phantom (64 tiles) gets 16 in both forms (FP64 in half-tile workgroups,
    two inline rows per tile), the 1024-tile EPI two, the 5e6-spin SE-EPI
    and the packed MRF batch one; a request for 1 or another valid count is
    honoured, others are rejected."""
    def info(k, prec="mixed", **kw):
        sc, ph, seq = W.config(k)
        return K.koma_plan_info(sc, ph, seq, K.make_config(prec, **kw))

    def lanes(k, prec="mixed", **kw):
        return info(k, prec, **kw)["lanes_per_spin"]
    assert lanes(1) == 16 and lanes(1, "fp64") == 16
    assert info(1)["n_rows"] == 64 and info(1, "fp64")["n_rows"] == 128
    assert info(1, "fp64", lanes_per_spin=8)["n_rows"] == 64
    assert lanes(2) == 2 and lanes(4) == 1
    assert lanes(1, lanes_per_spin=1) == 1 and lanes(1, lanes_per_spin=4) == 4
    with pytest.raises(K.KomaError):
        lanes(1, lanes_per_spin=3)
