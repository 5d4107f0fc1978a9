"""GPU parity of the HIP path (through the C-ABI) against the FP64 CPU oracle.

Tolerances (tests/_gpu.py, per signal row, normalised by its max|oracle|):
* KOMA_FP64: NRMSE and the largest sample error <= 1e-10. Differences come
  from rounding order, FMA contraction and the linear model of evenly spaced
  samples (measured ~1e-13).
* KOMA_MIXED: NRMSE and the largest sample error <= 1e-4 (the target
  accuracy), with the measured values printed; per dictionary entry for the
  MRF batch.
"""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W
from tests._gpu import TOL, case, check, errors, mae, nrmse, oracle_cached, say

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


def run(ctx, prec, key, **cfg):
    ctx.set_config(prec, **cfg)
    sc, ph, seq = case(key)
    return ctx.simulate(sc, ph, seq)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("key", ["gre", "epi_small", "mrf40", "seepi_subset"])
def test_parity_against_oracle(ctx, prec, key):
    say(f"[parity] {key} {prec}")
    ref = oracle_cached(key)
    got = run(ctx, prec, key)
    assert got.shape == ref.shape
    e = nrmse(got, ref)
    say(f"[parity] {key} {prec}: NRMSE median {float(np.median(e)):.3e}, "
        f"MAE {mae(got.ravel(), ref.ravel()):.3e}")
    check(got, ref, prec, f"parity {key}")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_parity_epi_full_size(ctx, prec):
    """The 256 x 256 head under the 128 x 128 single-shot EPI at full size,
    in the launch configuration the benchmark uses."""
    say(f"[parity] epi full {prec}")
    ref = oracle_cached("epi")
    got = run(ctx, prec, "epi")
    check(got, ref, prec, "parity epi full")


def test_closed_forms_on_gpu(ctx):
    """Hard pulse, FID and inversion recovery closed forms through the GPU path."""
    sc = W.Scanner()
    g = W.GAMMA
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        ctx.set_config(prec)
        # hard pulse in 7 pieces, T = inf
        tau, flip = 0.5e-3, 2.0
        t = np.linspace(0, tau, 8)
        seq = W.make_sequence(t, np.zeros((8, 3)), np.full(7, flip / (g * tau)), [7])
        s = ctx.simulate(sc, W.single_spin(pd=0.75), seq)[0, 0]
        assert abs(s - 1j * 0.75 * np.sin(flip)) < tol
        # FID
        tp, a = 2e-6, np.deg2rad(37.0)
        t = np.concatenate([[0, tp], tp + np.cumsum(np.full(50, 1e-3))])
        b1 = np.zeros(len(t) - 1, dtype=complex)
        b1[0] = a / (g * tp)
        ph = W.single_spin(pd=0.9, t1=0.8, t2=0.05)
        s = ctx.simulate(sc, ph, W.make_sequence(t, np.zeros((len(t), 3)), b1, np.arange(1, len(t))))[0]
        want = 1j * float(ph.pd[0]) * np.sin(a) * np.exp(-t[1:] / float(ph.t2[0]))
        assert np.max(np.abs(s - want)) < tol
        # inversion recovery read by m_final
        ti = 0.3
        t = np.array([0, 1e-6, ti])
        b1 = np.array([np.pi / (g * 1e-6), 0], dtype=complex)
        ph = W.single_spin(pd=1.0, t1=0.9, t2=0.1)
        _, m = ctx.simulate(sc, ph, W.make_sequence(t, np.zeros((3, 3)), b1, []), want_m=True)
        assert abs(m[0, 2] - (1 - 2 * np.exp(-ti / float(ph.t1[0])))) < tol


def test_magnitude_preserved_on_gpu(ctx):
    """T = inf: |M| = PD after ~10^4 random excitation steps. FP32 rounding of
    the four spinor coefficients and of the update moves |M| by ~6e-8 per step
    at random (no bias once the spinor is normalised with an exact defect), so
    after 10^4 steps the spread is ~6e-6 and the maximum over 300 spins stays
    below 5e-5; a biased step (e.g. a quantised normalisation) drifts ~1e-4."""
    rng = np.random.default_rng(7)
    seq = W.random_sequence(rng, 20_000, p_rf=0.5, p_adc=0.0)
    ph = W.random_spins(rng, 300, finite_t=False)
    for prec, tol in (("fp64", 1e-11), ("mixed", 5e-5)):
        ctx.set_config(prec)
        _, m = ctx.simulate(W.Scanner(), ph, seq, want_m=True)
        err = np.max(np.abs(np.linalg.norm(m, axis=1) / ph.pd - 1))
        say(f"[|M|] {prec}: max relative drift {err:.3e} over 20000 intervals (bar {tol:.0e})")
        assert err < tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_random_sequences_edge_cases(ctx, prec):
    """Random grids (non-uniform dt, RF and precession mixed, ADC at index 0,
    ADC right after RF, ADC on adjacent points), ragged spin counts and
    groups (including an empty group)."""
    import oracle
    rng = np.random.default_rng(11)
    sc = W.Scanner()
    for trial in range(4):
        seq = W.random_sequence(rng, int(rng.integers(50, 400)), p_rf=0.3, p_adc=0.6)
        seq.adc_idx = np.unique(np.concatenate([[0], seq.adc_idx]))
        n = int(rng.integers(1, 300))
        ph = W.random_spins(rng, n)
        cuts = np.sort(rng.integers(0, n + 1, 3))
        ph.group_off = np.concatenate([[0], cuts, [cuts[-1]], [n]])  # one empty group
        ref = oracle.simulate(sc, ph, seq)
        for dm, eng in ((-1, 0), (0, 0), (3, 0), (0, 1)):  # short stretches on both sample engines
            ctx.set_config(prec, defer_min_adc=dm, sample_engine=eng)
            got = ctx.simulate(sc, ph, seq)
            check(got, ref, prec, f"random grid {trial} defer {dm} engine {eng}")
    ctx.set_config(prec, defer_min_adc=32, sample_engine=0)


def _pulse_runs_sequence(with_gradient_rf=False):
    """Hard pulses of 1, 2, 3, 7, 50 and 1000 identical intervals, each
    followed by a gradient lobe and a few samples; optionally one pulse
    played under a gradient."""
    dt = 4e-6
    lens = (1, 2, 3, 7, 50, 1000)
    n_int = sum(lens) + len(lens) * 30 + (50 if with_gradient_rf else 0)
    s = W.UniformSeq(n_int, dt)
    p = 0
    for k, n in enumerate(lens):
        p = s.rf(p, W.hard_pulse(n, dt, (0.3 + 0.2 * k) * np.pi / 2))
        s.adc_points(p, 3)
        q = s.trap(0, p + 4, 3, 6, 2e-3 * (k + 1))
        s.adc_points(q, 4)
        p += 30
    if with_gradient_rf:
        s.trap(2, p - 1, 2, 38, 5e-3)   # Gz under the last pulse: intervals differ for moving spins
        p = s.rf(p, W.hard_pulse(40, dt, np.pi / 4))
    return s.build("pulse_runs")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_runs_of_identical_excitation_intervals(ctx, prec):
    """Runs of identical excitation intervals are applied by binary powering
    of one interval's affine map (rotation then relaxation): against the
    oracle's interval-by-interval steps, for spins with off-resonance (the
    per-spin spinor) and without (the precomputed zero-gradient rotation),
    with relaxation and with T = inf, and for moving spins."""
    import oracle
    rng = np.random.default_rng(31)
    sc = W.Scanner()
    seq = _pulse_runs_sequence()
    cases = [W.random_spins(rng, 200), W.random_spins(rng, 130, finite_t=False)]
    still = W.random_spins(rng, 128)
    still.dw[:] = 0.0                      # whole wavefronts without off-resonance
    cases.append(still)
    for ph in cases:
        ref = oracle.simulate(sc, ph, seq)
        ctx.set_config(prec)
        check(ctx.simulate(sc, ph, seq), ref, prec, f"excitation runs {ph.name}")
    mov_seq = _pulse_runs_sequence(with_gradient_rf=True)
    ph = W.with_velocity(W.random_spins(rng, 150), v=(0.05, -0.1, 0.2), spread=0.05)
    ref = oracle.simulate(sc, ph, mov_seq)
    check(ctx.simulate(sc, ph, mov_seq), ref, prec, "excitation runs, moving spins")
    say(f"[parity] excitation runs {prec}: ok")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_stretch_families_share_operands(ctx, prec):
    """Readout lines of three gradient amplitudes (3, 3 and 1 lines, in
    mixed order): the matrix-core kernel shares the per-sample operands
    within a family of equal increments; a stretch pair whose stretches
    belong to two families, and a short last batch, take their own paths.
    Several stretch lengths and tile counts per lane, both sample engines,
    and on the matrix cores batches of 4 and of 6 stretches per workgroup."""
    import oracle
    rng = np.random.default_rng(21)
    sc = W.Scanner()
    seq = W.readout_lines_sequence([0.01, -0.01, 0.01, 0.02, -0.01, 0.01, -0.01])
    ph = W.random_spins(rng, 300)
    ref = oracle.simulate(sc, ph, seq)
    for smax in (128, 16, 7):
        for spl in (1, 2, 8):
            for eng, ns in ((0, 4), (0, 6), (1, 0)):
                ctx.set_config(prec, spins_per_lane=spl, sample_engine=eng, stretch_max=smax, stretches_per_wg=ns)
                got = ctx.simulate(sc, ph, seq)
                e, m, z = errors(got, ref)
                assert z and e <= TOL[prec] and m <= TOL[prec], (smax, spl, eng, ns, e, m)
    say(f"[parity] stretch families {prec}: ok")
    ctx.set_config(prec, spins_per_lane=0, sample_engine=0, stretch_max=128, stretches_per_wg=0)


def test_random_readouts_every_engine_and_shape(ctx):
    """Seeded random cases: 1-8 readout lines of four amplitudes (so pairs of
    stretches of two families and short last batches occur), 8-199 samples
    per line, 1-699 spins in up to three groups, receive coils in some; each
    form on both sample engines with a random number of tiles per lane
    (1 .. 16, rounded down to 1, 2, 4 or 8 on the vector ALU), stretch
    length and stretches per matrix-core workgroup, against the oracle."""
    import oracle
    rng = np.random.default_rng(777)
    sc = W.Scanner()
    worst = {"fp64": 0.0, "mixed": 0.0}
    for trial in range(8):
        amps = list(rng.choice([0.01, -0.01, 0.02, -0.015], size=int(rng.integers(1, 9))))
        seq = W.readout_lines_sequence(amps, n_samples=int(rng.integers(8, 200)))
        n = int(rng.integers(1, 700))
        ph = W.random_spins(rng, n)
        if rng.random() < 0.5:
            cuts = np.sort(rng.integers(0, n + 1, 2))
            ph.group_off = np.concatenate([[0], cuts, [n]])
        if rng.random() < 0.3:
            ph = W.with_coils(ph, int(rng.integers(1, 4)))
        ref = oracle.simulate(sc, ph, seq)
        r2 = ref.reshape(-1, ref.shape[-1])
        mask = np.abs(r2).max(axis=1) > 0
        for prec in ("fp64", "mixed"):
            for eng in (0, 1):
                spl = int(rng.choice([0, 1, 2, 3, 5, 8, 16]))
                smax = int(rng.choice([128, 37, 16, 5]))
                ns = int(rng.choice([0, 4, 6]))
                ctx.set_config(prec, sample_engine=eng, spins_per_lane=spl, stretch_max=smax, stretches_per_wg=ns)
                got = ctx.simulate(sc, ph, seq).reshape(-1, ref.shape[-1])
                e, m, z = errors(got, r2)
                assert z, (trial, n, prec, eng)
                assert e <= TOL[prec] and m <= TOL[prec], (trial, n, prec, eng, spl, smax, ns, e, m)
                worst[prec] = max(worst[prec], m)
    ctx.set_config("mixed", sample_engine=0, spins_per_lane=0, stretch_max=128, stretches_per_wg=0)
    say(f"[parity] random readouts: worst max sample error fp64 {worst['fp64']:.2e}, mixed {worst['mixed']:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_launch_shape_invariance_and_determinism(ctx, prec):
    """Spins per lane and stretch length change only rounding; repeated runs
    are bitwise identical."""
    ref = oracle_cached("epi_small")
    outs = []
    for spl in (1, 2, 4, 8):
        for smax, ns in ((128, 4), (37, 4), (128, 6), (37, 6)):
            ctx.set_config(prec, spins_per_lane=spl, stretch_max=smax, stretches_per_wg=ns)
            sc, ph, seq = case("epi_small")
            a = ctx.simulate(sc, ph, seq)
            b = ctx.simulate(sc, ph, seq)
            assert np.array_equal(a, b)
            e, m, _ = errors(a, ref)
            assert e <= TOL[prec] and m <= TOL[prec], (spl, smax, ns, e, m)
            outs.append(a)
    ctx.set_config(prec, spins_per_lane=0, stretch_max=128, stretches_per_wg=0)


def test_device_pointers_match_host(ctx, K):
    import torch
    sc, ph, seq = case("epi_small")
    for prec in ("fp64", "mixed"):
        ctx.set_config(prec)
        host = ctx.simulate(sc, ph, seq)
        dph = K.device_phantom(ph)
        sig = torch.zeros((1, seq.n_adc, 2), dtype=torch.float64, device="cuda:0")
        ctx.simulate(sc, dph, seq, where="device", sig=sig)
        dev = sig.cpu().numpy()
        assert np.array_equal(dev[..., 0] + 1j * dev[..., 1], host)


def test_request_path_equals_simulate(ctx):
    """Chunked execution with device-resident state gives the same bits as
    one whole simulation, for any chunk length, and survives a checkpoint.
    With one lane per spin the chunks also start and end inside the runs of
    single excitation intervals of the GRE sinc pulses, on both sides of the
    64-event LDS stage."""
    sc, ph, seq = case("gre")
    ph = ph.subset(np.arange(1000))
    for prec in ("fp64", "mixed"):
        for lanes, chunks in ((1, (1, 63, 64, 65, 97, 100000)), (0, (1, 97, 100000))):
            ctx.set_config(prec, lanes_per_spin=lanes)
            whole = ctx.simulate(sc, ph, seq)
            for chunk in chunks:
                r = ctx.open(sc, ph, seq)
                while not r.done():
                    r.advance(chunk)
                assert np.array_equal(r.result(), whole), (prec, lanes, chunk)
                r.close()
        # checkpoint half way (the planner's lanes per spin, as the last whole
        # run), restore into a fresh request
        r = ctx.open(sc, ph, seq)
        for _ in range(30):
            r.advance(100)
        blob = r.save()
        r2 = ctx.open(sc, ph, seq)
        r2.load(blob)
        r.close()
        while not r2.done():
            r2.advance(500)
        assert np.array_equal(r2.result(), whole)
        r2.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_one_lane_per_spin_runs_against_oracle(ctx, prec):
    """One lane per spin on the SE-EPI subset: the 100- and 200-interval sinc
    pulses are runs of single intervals longer than the 64-event LDS stage,
    taken by the run loop in pieces; against the oracle."""
    say(f"[parity] seepi_subset one lane {prec}")
    ref = oracle_cached("seepi_subset")
    ctx.set_config(prec, lanes_per_spin=1)
    sc, ph, seq = case("seepi_subset")
    check(ctx.simulate(sc, ph, seq), ref, prec, "seepi subset, one lane per spin")
    ctx.set_config(prec)


def test_invalid_device_phantom_is_rejected(ctx, K):
    import torch
    sc, ph, seq = case("epi_small")
    dph = K.device_phantom(ph)
    dph["t2"][5] = float("nan")
    sig = torch.full((1, seq.n_adc, 2), -3.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(K.KomaError) as e:
        ctx.simulate(sc, dph, seq, where="device", sig=sig)
    assert e.value.status == -2
    assert bool(torch.all(sig == -3.0))  # the output is left untouched
    # the context still works afterwards
    assert np.isfinite(ctx.simulate(sc, ph, seq)).all()


def test_precomputed_zero_gradient_rotation_matches_general_path(ctx):
    """Zero-gradient excitation intervals of wavefronts without off-resonance
    use a rotation precomputed on the host; spins with a negligible (but not
    zero) off-resonance take the per-spin spinor path. Both must agree, and
    both must match the oracle."""
    import oracle
    sc, ph, seq = case("mrf40")
    ph2 = W.Phantom(ph.x, ph.y, ph.z, ph.pd, ph.t1, ph.t2, np.full(ph.n, 1e-30), ph.group_off)
    ref = oracle_cached("mrf40")
    for prec, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        ctx.set_config(prec)
        fast = ctx.simulate(sc, ph, seq)
        slow = ctx.simulate(sc, ph2, seq)
        e = float(np.max(nrmse(fast, slow)))
        say(f"[rot] {prec}: fast vs per-spin path NRMSE {e:.3e}; vs oracle "
            f"{float(np.max(nrmse(fast, ref))):.3e} / {float(np.max(nrmse(slow, ref))):.3e}")
        assert e <= tol
        check(fast, ref, prec, "zero-gradient rotation, precomputed")
        check(slow, ref, prec, "zero-gradient rotation, per-spin spinor")


def test_magnitude_preserved_by_repeated_hard_pulses(ctx):
    """T = inf, no gradient, no off-resonance: 10^4 excitation intervals of
    varying flip (the precomputed-rotation path) keep |M| = PD."""
    rng = np.random.default_rng(17)
    n = 10_000
    dt = rng.uniform(1e-6, 1e-5, n)
    t = np.concatenate([[0.0], np.cumsum(dt)])
    b1 = rng.uniform(-2e-5, 2e-5, n) + 1j * rng.uniform(-2e-5, 2e-5, n)
    seq = W.make_sequence(t, np.zeros((n + 1, 3)), b1, [])
    ph = W.random_spins(rng, 200, finite_t=False)
    ph.dw[:] = 0
    for prec, tol in (("fp64", 1e-11), ("mixed", 5e-5)):
        ctx.set_config(prec)
        _, m = ctx.simulate(W.Scanner(), ph, seq, want_m=True)
        err = np.max(np.abs(np.linalg.norm(m, axis=1) / ph.pd - 1))
        say(f"[|M| hard] {prec}: max relative drift {err:.3e} over {n} intervals")
        assert err < tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("which", ["gre", "epi_small"])
def test_minimal_grid_on_gpu_matches_raster_oracle(ctx, K, prec, which):
    """Sequence-aware time stepping end to end: the library discretises the
    block form of the sequence to its minimal grid (gradient vertices, RF
    samples, ADC points only) and the GPU simulates it; the result matches
    the oracle on the same minimal grid at the parity bar, and the oracle on
    the raster grid of the same sequence within the bound of two FP64 phase
    sums over different grids (64 eps x the largest accumulated phase, the
    bound the discretiser's own pin uses) in the FP64 form, at the mixed bar
    in the mixed form."""
    import oracle
    from tests.test_discretize import phase_scale
    sc, ph, ref_seq = case(which)
    blocks = W.gre_blocks() if which == "gre" else W.epi_blocks(n=64, ramp=8)
    m = K.koma_discretize(blocks)
    assert m.n_adc == ref_seq.n_adc and m.n_int < ref_seq.n_int
    ref_raster = oracle_cached(which)
    ref_min = oracle.simulate(sc, ph, m, mode=oracle.MODE_BLOCK)
    ctx.set_config(prec)
    got = ctx.simulate(sc, ph, m)
    say(f"[minimal grid] {which} {prec}: {m.n_int} vs {ref_seq.n_int} intervals")
    check(got, ref_min, prec, f"minimal grid {which} vs oracle on the minimal grid")
    if prec == "fp64":
        bound = 64 * np.finfo(float).eps * phase_scale(ref_seq, ph)
        e = float(np.max(nrmse(got, ref_raster)))
        say(f"[minimal grid] {which}: NRMSE vs raster oracle {e:.3e} (grid bound {bound:.2e})")
        assert e < bound
    else:
        check(got, ref_raster, prec, f"minimal grid {which} vs raster oracle")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("key", ["epi_small", "gre", "seepi_subset"])
def test_sample_engines_agree(ctx, key, prec):
    """The deferred sample sums on the matrix cores (FP32 MFMA in the mixed
    form, FP64 MFMA in the FP64 form) and on the vector ALU: both within the
    parity bar of the oracle and of each other."""
    ref = oracle_cached(key)
    out = {}
    for eng in (0, 1):
        ctx.set_config(prec, sample_engine=eng)
        sc, ph, seq = case(key)
        out[eng] = ctx.simulate(sc, ph, seq)
    ctx.set_config(prec, sample_engine=0)
    check(out[0], ref, prec, f"engine {key} matrix cores")
    check(out[1], ref, prec, f"engine {key} vector ALU")
    check(out[0], out[1], prec, f"engine {key} matrix cores vs vector ALU")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_packed_tiles_match_oracle(ctx, prec):
    """Wavefronts across signal-group boundaries (packed tiles) sum each
    group's lanes apart: the 40-entry MRF batch (400-spin groups) packed and
    per group, and through the chunked request path; random groups of >= 64
    spins with empty groups among them, with and without receive coils."""
    import oracle
    ref = oracle_cached("mrf40")
    sc, ph, seq = case("mrf40")
    out = {}
    for packing in (1, 0):
        ctx.set_config(prec, tile_packing=packing)
        out[packing] = ctx.simulate(sc, ph, seq)
        check(out[packing], ref, prec, f"mrf40 tile packing {packing}")
    ctx.set_config(prec, tile_packing=1)
    r = ctx.open(sc, ph, seq)
    while not r.done():
        r.advance(333)
    assert np.array_equal(r.result(), out[1])
    r.close()
    rng = np.random.default_rng(61)
    sizes = rng.integers(64, 200, 12)
    sizes[[2, 7]] = 0
    off = np.concatenate([[0], np.cumsum(sizes)])
    sp = W.random_spins(rng, int(off[-1]))
    sp.group_off = off
    rseq = W.random_sequence(rng, 200, p_rf=0.3, p_adc=0.5)
    for n_coils in (0, 3):
        phx = W.with_coils(sp, n_coils) if n_coils else sp
        ref = oracle.simulate(sc, phx, rseq)
        for packing in (1, 0):
            ctx.set_config(prec, tile_packing=packing, defer_min_adc=-1)
            check(ctx.simulate(sc, phx, rseq), ref, prec, f"random groups, {n_coils} coils, packing {packing}")
    ctx.set_config(prec, tile_packing=1, defer_min_adc=32)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_several_lanes_per_spin_match_oracle(ctx, prec):
    """Several lanes per spin: each lane composes the affine maps of a share
    of every segment of excitation intervals and block ends, the lanes'
    products are combined and applied. Every lane count against the oracle
    on the GRE workload (sinc excitations, one lane per spin otherwise
    latency-bound), random grids with inline samples, several signal groups,
    coils and moving spins (FP64 at 16 lanes runs half-tile workgroups, each
    with its own inline rows); the chunked request path (chunks end at
    segment ends) gives the bits of one whole run."""
    import oracle
    sc, ph, seq = case("gre")
    ref = oracle_cached("gre")
    lanes = (1, 2, 4, 8, 16)
    for g in lanes:
        ctx.set_config(prec, lanes_per_spin=g)
        check(ctx.simulate(sc, ph, seq), ref, prec, f"gre, {g} lanes per spin")
    rng = np.random.default_rng(71)
    for trial in range(3):
        rseq = W.random_sequence(rng, int(rng.integers(100, 500)), p_rf=0.5, p_adc=0.2)
        sp = W.random_spins(rng, int(rng.integers(1, 200)))
        if trial == 0 and sp.n >= 3:
            sp.group_off = np.array([0, sp.n // 3, sp.n // 3, sp.n])  # an empty group among three
        if trial == 1:
            sp = W.with_coils(sp, 2)
        if trial == 2:
            sp = W.with_velocity(sp, rng.uniform(-0.3, 0.3, 3), spread=0.2, seed=3)
        rref = oracle.simulate(sc, sp, rseq)
        for g in lanes:
            for dm in (-1, 32):
                ctx.set_config(prec, lanes_per_spin=g, defer_min_adc=dm)
                check(ctx.simulate(sc, sp, rseq), rref, prec, f"random grid {trial}, {g} lanes, defer {dm}")
    ph1 = ph.subset(np.arange(700))
    for g in lanes[1:]:
        ctx.set_config(prec, lanes_per_spin=g)
        whole = ctx.simulate(sc, ph1, seq)
        for chunk in (1, 37, 1000):
            r = ctx.open(sc, ph1, seq)
            while not r.done():
                r.advance(chunk)
            assert np.array_equal(r.result(), whole), (g, chunk)
            r.close()
    ctx.set_config(prec, lanes_per_spin=0, defer_min_adc=32)


def test_random_configurations_against_oracle(ctx):
    """Seeded random cases (readout lines or random grids, 1-1,499 spins in
    up to four groups, receive coils, moving spins) under random settings of
    every planner knob (sample engine, tiles per wavefront, stretch length,
    stretches per matrix-core workgroup, lanes per spin, deferral threshold,
    tile packing), both forms, against the oracle."""
    import oracle
    rng = np.random.default_rng(777)
    sc = W.Scanner()
    worst = {"fp64": 0.0, "mixed": 0.0}
    for trial in range(60):
        if rng.random() < 0.5:
            amps = list(rng.choice([0.01, -0.01, 0.02, -0.015, 0.005], size=int(rng.integers(1, 12))))
            seq = W.readout_lines_sequence(amps, n_samples=int(rng.integers(4, 260)))
        else:
            seq = W.random_sequence(rng, int(rng.integers(20, 600)), p_rf=float(rng.uniform(0.1, 0.7)),
                                    p_adc=float(rng.uniform(0.05, 0.5)))
        n = int(rng.integers(1, 1500))
        ph = W.random_spins(rng, n)
        if rng.random() < 0.5 and n >= 3:
            cuts = np.sort(rng.integers(0, n + 1, int(rng.integers(1, 4))))
            ph.group_off = np.concatenate([[0], cuts, [n]])
        if rng.random() < 0.25:
            ph = W.with_coils(ph, int(rng.integers(1, 4)))
        if rng.random() < 0.2:
            ph = W.with_velocity(ph, rng.uniform(-0.3, 0.3, 3), spread=0.2, seed=int(rng.integers(1, 1000)))
        ref = oracle.simulate(sc, ph, seq)
        for prec in ("fp64", "mixed"):
            cfg = dict(sample_engine=int(rng.integers(0, 2)),
                       spins_per_lane=int(rng.choice([0, 1, 2, 3, 5, 8, 11, 16])),
                       stretch_max=int(rng.choice([128, 64, 37, 16, 5, 1])),
                       stretches_per_wg=int(rng.choice([0, 4, 6])),
                       lanes_per_spin=int(rng.choice([0, 1, 2, 4, 8, 16])),
                       defer_min_adc=int(rng.choice([-1, 1, 8, 32])),
                       tile_packing=int(rng.integers(0, 2)))
            ctx.set_config(prec, **cfg)
            e, m, z = errors(ctx.simulate(sc, ph, seq), ref)
            assert z and e <= TOL[prec] and m <= TOL[prec], (trial, n, prec, cfg, e, m)
            worst[prec] = max(worst[prec], m)
    ctx.set_config("mixed", sample_engine=0, spins_per_lane=0, stretch_max=128, stretches_per_wg=0,
                   lanes_per_spin=0, defer_min_adc=32, tile_packing=1)
    say(f"[parity] random configurations: worst max sample error fp64 {worst['fp64']:.2e}, mixed {worst['mixed']:.2e}")
