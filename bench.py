#!/usr/bin/env python3
"""Benchmark of the Bloch-simulation hot path on one MI355X.

Headline: the large 2D multi-slice spin-echo EPI (5e6 spins in 20 slices
of 500 x 500; per slice a 100-interval sinc 90 deg, a 200-interval sinc
180 deg and a 128 x 128 EPI readout with k_y = 0 at TE = 60 ms; dt = 4 us,
563,900 intervals, 327,680 ADC samples), the largest configuration of the
measured set that one GPU holds. A step is one whole simulation through
``koma_simulate_async``: host packing of the sequence into the event
program, its upload, every kernel, with the phantom and the signal in HBM.
``value`` is grid spin-steps per second (spins x intervals / time) of the
mixed-precision form; beside it in the same JSON line: the all-FP64 form,
events/s, the roofline of every kernel of the step (the dominant one as
``roofline``), the error against the FP64 oracle, the oracle's own CPU rate
on a seeded spin subset, the other workloads (each with its error against
the oracle), the sequence-aware grids, motion and coils, MRF dictionary
matching, and the serving figures.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G spin-steps/s (mixed vs FP64 GPU) + serving p50/p99 latency at NRMSE<=1e-4"
# Published MI355X peaks
PEAK_FP32 = 157.3      # TFLOP/s FP32 (vector / dense matrix); the vector figure holds without packed
                       # instructions too: a 32-bit-encoded FP32 instruction issues at about two cycles
                       # per wave64 (measured), 256 CU x 4 SIMD x 32 lanes x 2 FLOP x 2.4 GHz
PEAK_FP64 = 78.6       # TFLOP/s FP64 (vector and dense matrix)
PEAK_HBM = 8000.0      # GB/s
PEAK_FP16 = 2500.0     # TFLOP/s dense FP16 matrix
# Algorithmic work per unit (see the measurement section of the design notes)
FLOP_PER_TERM = 8      # (spin, sample) of a deferred block: complex multiply (6) + add (2)
FLOP_PER_RF = 65       # (spin, excitation interval): field, spinor, Eq. Rot_exc, relaxation
FLOP_PER_END = 17      # (spin, block end): FP64 phase (8), complex rotate (6), Mz relaxation (3)
FLOP_PER_INLINE = 8    # (spin, inline sample): factor (6) + accumulate (2)
TRANS_PER_RF = 3       # rsqrt, sin, cos
TRANS_PER_END = 3      # sin, cos, exp


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(files=("komahip_kernels.hip", "komahip_internal.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2301_02702_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def err(got, ref):
    """(NRMSE, max sample error, MAE), each over rows of the last axis and
    normalised by the row's max|ref|; the worst row."""
    r = np.asarray(ref).reshape(-1, np.shape(ref)[-1])
    g = np.asarray(got).reshape(r.shape)
    s = np.max(np.abs(r), axis=1)
    nz = s > 0
    d = np.abs(g - r)[nz]
    return {"nrmse": float(np.max(np.sqrt(np.mean(d ** 2, axis=1)) / s[nz])),
            "max_err": float(np.max(np.max(d, axis=1) / s[nz])),
            "mae": float(np.max(np.mean(d, axis=1) / s[nz]))}


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


_STREAM = []


def _bench_stream(torch):
    if not _STREAM:
        _STREAM.append(torch.cuda.Stream())
    return _STREAM[0]


def run_workload(K, ctx, torch, sc, ph, seq, prec, steps, warmup, profile_steps=0, pipelined=False):
    """Time `steps` device-resident simulations; return (seconds per step, signal, kernel stats).

    A step is one whole simulation: host packing of the sequence, upload of
    the packed tables, every kernel. Synchronous: koma_simulate, which waits
    for its stream (the latency of one call). Pipelined: koma_simulate_async
    on one stream, so the host packs step k + 1 while the device runs step k
    (the throughput of a stream of simulations). Kernel statistics come from
    a separate profiled pass of `profile_steps` steps (the profiler records
    HIP events around every launch on the stream it is launched on, which is
    kept out of the timed steps)."""
    ctx.set_config(prec)
    dph = K.device_phantom(ph)
    nsig = getattr(ph, "n_coils", 0) or 1
    sig = torch.zeros((nsig, ph.n_groups, seq.n_adc, 2), dtype=torch.float64, device="cuda:0")
    # a stream of its own (default priority): launches on the legacy default
    # stream synchronise with the other blocking streams of the process
    stream = _bench_stream(torch)
    torch.cuda.synchronize()  # the phantom and the signal buffer are made on the default stream
    if pipelined:
        step = ctx.bind_async(sc, dph, seq, sig, stream=stream)
    else:
        def step():
            ctx.simulate(sc, dph, seq, where="device", sig=sig, stream=stream)
    t = time_steps(step, steps, warmup, torch)
    stats = None
    if profile_steps:
        ctx.profile(True)
        time_steps(step, profile_steps, 0, torch)
        stats = {k: ctx.kernel_stats(k) for k in ("seq", "par", "reduce", "aux")}
        stats["steps"] = profile_steps
        ctx.profile(False)
    s = sig.cpu().numpy()
    out = s[..., 0] + 1j * s[..., 1]
    del dph, sig
    return t, (out if nsig > 1 else out[0]), stats


def per_launch(st, kind):
    k = st[kind]
    return k["total_ms"] / max(k["launches"], 1), k["launches"] / st["steps"]


def rooflines(info, st, prec, n_spins, traffic=None):
    """Roofline of every kernel of a step from the live HIP-event timing.
    Units and per-unit work: the measurement section of the design notes.
    ``traffic``: stored HBM bytes per launch by kernel (rocprofv3 counters of
    the same kernels), turned into GB/s with the live launch times."""
    out = {}
    fp64 = prec == "fp64"
    # sample-parallel sums: dense contraction on the matrix cores
    if st["par"]["launches"]:
        ms, lps = per_launch(st, "par")
        units = n_spins * info["n_deferred_adc"]
        ach = FLOP_PER_TERM * units / lps / (ms * 1e-3) / 1e12
        peak = PEAK_FP64 if fp64 else PEAK_FP32
        out["k_par_mm64" if fp64 else "k_par_mm"] = {
            "bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 4), "avg_launch_ms": round(ms, 5), "launches_per_step": lps,
            "flop_per_unit": FLOP_PER_TERM, "units_per_step": units,
            "unit_def": "one (spin, ADC sample) term of a deferred precession block",
            "peak_def": "FP64 dense matrix" if fp64 else "FP32 dense matrix"}
    # spin-sequential kernel: vector ALU
    if st["seq"]["launches"]:
        ms, lps = per_launch(st, "seq")
        rf_single = info["n_rf_events"] - (info["n_runs"] if info["n_rf_in_runs"] else 0)
        flop = n_spins * (FLOP_PER_RF * info["n_rf_events"] + FLOP_PER_END * info["n_ends"]
                          + FLOP_PER_INLINE * info["n_inline_adc"])
        trans = n_spins * (TRANS_PER_RF * info["n_rf_events"] + TRANS_PER_END * info["n_ends"])
        ach = flop / lps / (ms * 1e-3) / 1e12
        peak = PEAK_FP64 if fp64 else PEAK_FP32
        out["k_seq"] = {
            "bound": "alu", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 4),
            "transcendentals_per_s": round(trans / lps / (ms * 1e-3), 1),
            "avg_launch_ms": round(ms, 5), "launches_per_step": lps, "flop_per_step": flop,
            "units": {"excitation_event": [FLOP_PER_RF, info["n_rf_events"]], "block_end": [FLOP_PER_END, info["n_ends"]],
                      "inline_sample": [FLOP_PER_INLINE, info["n_inline_adc"]]},
            "single_interval_events": rf_single,
            "peak_def": "FP64 vector" if fp64 else "FP32 vector"}
    # fixed-order FP64 sums of the workgroup partials: HBM
    if st["reduce"]["launches"]:
        ms, lps = per_launch(st, "reduce")
        out["k_reduce"] = {"bound": "hbm", "avg_launch_ms": round(ms, 5), "launches_per_step": lps}
    if traffic:
        for name, r in out.items():
            key = f"{name}:{prec}"
            if key in traffic.get("kernels", {}):
                b = traffic["kernels"][key]["bytes_per_launch"]
                r["traffic"] = b
                r["hbm_GBps"] = round(b / (r["avg_launch_ms"] * 1e-3) / 1e9, 2)
                r["hbm_frac"] = round(r["hbm_GBps"] / PEAK_HBM, 5)
                r["traffic_source"] = traffic["source"]
        if "k_reduce" in out and "hbm_GBps" in out["k_reduce"]:
            out["k_reduce"].update(achieved=out["k_reduce"]["hbm_GBps"], peak=PEAK_HBM, unit="GB/s",
                                   frac=out["k_reduce"]["hbm_frac"])
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sc, ph, seq, n_multi, n_single, seed=5050):
    """The oracle (per-interval FP64 splitting, as it stands) on seeded spin
    subsets of the workload: n_multi spins on every thread the process may
    use (at most 16, the host share of one GPU), n_single spins on one
    thread. Returns (subset index, oracle signal of the multi-thread subset,
    report)."""
    import oracle
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(ph.n, n_multi, replace=False))
    sub = ph.subset(idx)
    th = oracle.default_threads()
    t0 = time.perf_counter()
    ref = oracle.simulate(sc, sub, seq, mode=oracle.MODE_STEP, threads=th)
    dt = time.perf_counter() - t0
    sub1 = ph.subset(idx[:n_single])
    t0 = time.perf_counter()
    oracle.simulate(sc, sub1, seq, mode=oracle.MODE_STEP, threads=1)
    dt1 = time.perf_counter() - t0
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count()
    rep = {"value": round(n_multi * seq.n_int / dt / 1e9, 4), "unit": "G spin-steps/s", "cores": th,
           "kind": "oracle", "wall_s": round(dt, 3),
           "sample": f"{n_multi} seeded spins of the {ph.n} (all slices) x the full {seq.n_int}-interval "
                     "sequence, per-interval FP64 splitting, one signal matrix per thread",
           "one_thread": {"value": round(n_single * seq.n_int / dt1 / 1e9, 5), "wall_s": round(dt1, 3),
                          "sample": f"the first {n_single} spins of that subset"},
           "cpu_model": cpu_model(), "cpus_available": avail}
    return idx, ref, rep


def load_stored(name, khash):
    """A counter figure taken by rocprofv3 and committed under profiles/ with
    the kernel source hash it was taken with; None once the kernels changed."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_hash") != khash:
        return None
    d["source"] = f"stored: profiles/{name}"
    return d


def oracle_entries(sc, ph, seq, entries):
    import oracle
    return np.stack([oracle.simulate(sc, ph.groups(int(e), int(e) + 1), seq, mode=oracle.MODE_BLOCK)[0]
                     for e in entries])


def bench_headline(K, ctx, torch, W, args, khash):
    sc, ph, seq = W.config(5)
    info = K.koma_plan_info(sc, ph, seq, K.make_config("mixed"))
    spin_steps = ph.n * seq.n_int
    prof = min(args.steps, 5)
    log(f"[bench] headline seepi: {ph.n} spins x {seq.n_int} intervals, {seq.n_adc} ADC")
    t_mix, s_mix, st_mix = run_workload(K, ctx, torch, sc, ph, seq, "mixed", args.steps, args.warmup, prof, True)
    log(f"[bench] seepi mixed, pipelined: {t_mix * 1e3:.2f} ms/step")
    t_64, s_64, st_64 = run_workload(K, ctx, torch, sc, ph, seq, "fp64", args.steps, args.warmup, prof, True)
    log(f"[bench] seepi fp64, pipelined: {t_64 * 1e3:.2f} ms/step")
    events = ph.n * (info["n_rf_events"] + info["n_ends"] + info["n_adc"])
    traffic = load_stored("traffic_seepi.json", khash)
    rl_mix = rooflines(info, st_mix, "mixed", ph.n, traffic)
    rl_64 = rooflines(info, st_64, "fp64", ph.n, traffic)
    kms = {p: {k: round(v["total_ms"] / st["steps"], 3) for k, v in st.items() if k != "steps"}
           for p, st in (("mixed", st_mix), ("fp64", st_64))}
    dom = max(("k_par_mm", "par"), ("k_seq", "seq"), key=lambda kv: kms["mixed"][kv[1]])[0]
    roofline = dict(rl_mix[dom], kernel=dom)
    roofline.setdefault("traffic", None)
    flops = load_stored("flops_seepi.json", khash)
    out = {
        "metric": METRIC, "value": round(spin_steps / t_mix / 1e9, 3), "unit": "G spin-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_mix * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "seepi20x500_mixed: multi-slice spin-echo EPI, 5e6 spins (20 slices of "
                               "500x500 seeded head phantoms, 100 Hz smooth off-resonance), per slice sinc 90 "
                               "(100 int) + sinc 180 (200 int) + 128x128 EPI readout, TE 60 ms, dt 4 us, "
                               f"{seq.n_int} intervals, {seq.n_adc} ADC samples",
                   "spins": ph.n, "intervals": seq.n_int, "adc": seq.n_adc, "spin_steps": spin_steps,
                   "phantom_in": "HBM", "signal_out": "HBM", "sequence_packing": "host, every step",
                   "steps": "pipelined: koma_simulate_async on one stream"},
        "fp64": {"value": round(spin_steps / t_64 / 1e9, 3), "ms_per_step": round(t_64 * 1e3, 4),
                 "roofline": rl_64},
        "mixed_over_fp64": round(t_64 / t_mix, 3),
        "events_per_s": {"mixed": round(events / t_mix, 1), "fp64": round(events / t_64, 1),
                         "events_per_spin": info["n_rf_events"] + info["n_ends"] + info["n_adc"],
                         "def": "per spin: excitation events + block ends + ADC samples evaluated"},
        "kernel_ms_per_step": kms,
        "roofline": roofline,
        "rooflines": {"mixed": rl_mix, "fp64": rl_64},
        "rocprof_flops": flops,
    }
    # error against the FP64 oracle: the oracle on a seeded spin subset (the
    # CPU baseline run); FP64 by linearity at full size (full - rest =
    # subset); mixed on the subset directly and against FP64 at full size
    out["nrmse_mixed_vs_fp64"] = err(s_mix, s_64)
    if not args.no_cpu:
        log("[bench] oracle CPU baseline on a seeded subset of the seepi spins ...")
        idx, ref, cpu = cpu_baseline(sc, ph, seq, args.cpu_spins, args.cpu_spins_1t)
        out["cpu_baseline"] = cpu
        log(f"[bench] oracle {cpu['wall_s']} s on {cpu['cores']} threads ({cpu['value']} G spin-steps/s); "
            f"1 thread {cpu['one_thread']['value']}")
        keep = np.ones(ph.n, dtype=bool)
        keep[idx] = False
        rest = ph.subset(np.nonzero(keep)[0])
        _, s_rest, _ = run_workload(K, ctx, torch, sc, rest, seq, "fp64", 1, 0)
        del rest
        sub = ph.subset(idx)
        _, s_sub_mix, _ = run_workload(K, ctx, torch, sc, sub, seq, "mixed", 1, 0)
        _, s_sub_64, _ = run_workload(K, ctx, torch, sc, sub, seq, "fp64", 1, 0)
        out["error_vs_oracle"] = {
            "fp64_full_size_by_linearity": err(s_64 - s_rest, ref),
            "fp64_subset": err(s_sub_64, ref), "mixed_subset": err(s_sub_mix, ref),
            "subset_spins": int(len(idx)),
            "def": "oracle on the seeded subset; fp64_full_size_by_linearity = FP64(all spins) - "
                   "FP64(all but the subset) against it; *_subset = the GPU run on the subset alone"}
        log(f"[bench] seepi error vs oracle: {out['error_vs_oracle']}")
    else:
        out["cpu_baseline"] = None
    return out


def bench_secondary(K, ctx, torch, W, args, out):
    import oracle
    # epi256: the 256 x 256 head, 128 x 128 single-shot EPI (65,536 spins)
    sc, ph, seq = W.config(2)
    ss = ph.n * seq.n_int
    info = K.koma_plan_info(sc, ph, seq, K.make_config("mixed"))
    t_m, s_m, st_m = run_workload(K, ctx, torch, sc, ph, seq, "mixed", args.epi_steps, 20, 50, True)
    t_m1, _, _ = run_workload(K, ctx, torch, sc, ph, seq, "mixed", args.epi_steps, 20)
    t_6, s_6, st_6 = run_workload(K, ctx, torch, sc, ph, seq, "fp64", args.epi_steps, 20, 50, True)
    ctx.set_config("mixed", sample_engine=1)  # the same sums on the vector ALU, for comparison
    t_v, s_v, st_v = run_workload(K, ctx, torch, sc, ph, seq, "mixed", args.epi_steps, 20, 50, True)
    ctx.set_config("mixed", sample_engine=0)
    ref = oracle.simulate(sc, ph, seq, mode=oracle.MODE_BLOCK)[0]
    rl_m = rooflines(info, st_m, "mixed", ph.n)
    par_v, lps_v = per_launch(st_v, "par")
    ach_v = FLOP_PER_TERM * ph.n * info["n_deferred_adc"] / lps_v / (par_v * 1e-3) / 1e12
    w = {"spins": ph.n, "intervals": seq.n_int, "spin_steps": ss,
         "mixed_gsps": round(ss / t_m / 1e9, 3), "mixed_ms": round(t_m * 1e3, 4),
         "mixed_one_call_ms": round(t_m1 * 1e3, 4),
         "fp64_gsps": round(ss / t_6 / 1e9, 3), "fp64_ms": round(t_6 * 1e3, 4),
         "rooflines": {"mixed": rl_m, "fp64": rooflines(info, st_6, "fp64", ph.n)},
         "mixed_valu_sums": {"ms": round(t_v * 1e3, 4), "par_ms": round(par_v, 5),
                             "roofline": {"bound": "alu", "kernel": "k_par (vector ALU)",
                                          "achieved": round(ach_v, 3), "peak": PEAK_FP32,
                                          "frac": round(ach_v / PEAK_FP32, 4)},
                             "vs_mfma": err(s_v, s_m)},
         "error_vs_oracle": {"mixed": err(s_m, ref), "fp64": err(s_6, ref)}}
    log(f"[bench] epi256: mixed {w['mixed_gsps']}, fp64 {w['fp64_gsps']} G spin-steps/s; vs oracle "
        f"{w['error_vs_oracle']}")
    wl = {"epi256": w}
    dictionary = None
    # gre64 (whole oracle) and the MRF batch (oracle on 48 seeded entries)
    for k in (1, 4):
        sck, phk, seqk = W.config(k)
        ss = phk.n * seqk.n_int
        infok = K.koma_plan_info(sck, phk, seqk, K.make_config("mixed"))
        # a stream of simulations (pipelined) and one call at a time
        n_pipe = 40 if k == 1 else 10
        tm, sm, km = run_workload(K, ctx, torch, sck, phk, seqk, "mixed", n_pipe, 2, 3, True)
        t6, s6, k6 = run_workload(K, ctx, torch, sck, phk, seqk, "fp64", n_pipe, 2, 3, True)
        tm1, _, _ = run_workload(K, ctx, torch, sck, phk, seqk, "mixed", 5, 1)
        t61, _, _ = run_workload(K, ctx, torch, sck, phk, seqk, "fp64", 5, 1)
        name = W.WORKLOAD_NAMES[k].split(" ")[0]
        w = {"spins": phk.n, "intervals": seqk.n_int, "spin_steps": ss,
             "mixed_gsps": round(ss / tm / 1e9, 3), "fp64_gsps": round(ss / t6 / 1e9, 3),
             "mixed_ms": round(tm * 1e3, 3), "fp64_ms": round(t6 * 1e3, 3),
             "mixed_one_call_ms": round(tm1 * 1e3, 3), "fp64_one_call_ms": round(t61 * 1e3, 3),
             "timing": "ms: pipelined stream of koma_simulate_async calls; one_call_ms: koma_simulate, synchronous",
             "events_per_spin": infok["n_rf_events"] + infok["n_ends"] + infok["n_adc"],
             "kernel_ms": {p: {kk: round(v["total_ms"] / st["steps"], 3) for kk, v in st.items() if kk != "steps"}
                           for p, st in (("mixed", km), ("fp64", k6))},
             "rooflines": {"mixed": rooflines(infok, km, "mixed", phk.n), "fp64": rooflines(infok, k6, "fp64", phk.n)}}
        if k == 1:
            ref = oracle.simulate(sck, phk, seqk, mode=oracle.MODE_BLOCK)
            w["error_vs_oracle"] = {"mixed": err(sm, ref), "fp64": err(s6, ref)}
        else:
            dictionary = sm.astype(np.complex64)  # 10,000 simulated fingerprints x 1,000 TRs
            rng = np.random.default_rng(4004)
            entries = np.sort(rng.choice(phk.n_groups, 48, replace=False))
            ref = oracle_entries(sck, phk, seqk, entries)
            per = {}
            for p, s in (("mixed", sm), ("fp64", s6)):
                d = np.abs(s[entries] - ref)
                sc_ = np.max(np.abs(ref), axis=1)
                e = np.sqrt(np.mean(d ** 2, axis=1)) / sc_
                worst = int(np.argmax(e))
                per[p] = {"nrmse_max": float(e.max()), "nrmse_p99": float(np.percentile(e, 99)),
                          "nrmse_median": float(np.median(e)),
                          "max_err": float(np.max(np.max(d, axis=1) / sc_)),
                          "worst_entry_t1_t2": [float(phk.t1[phk.group_off[entries[worst]]]),
                                                float(phk.t2[phk.group_off[entries[worst]]])]}
            w["error_vs_oracle_per_entry"] = dict(per, entries=48)
            e = np.sqrt(np.mean(np.abs(sm - s6) ** 2, axis=1)) / np.max(np.abs(s6), axis=1)
            w["nrmse_mixed_vs_fp64_all_entries"] = {"max": float(e.max()), "median": float(np.median(e))}
        log(f"[bench] {name}: mixed {w['mixed_gsps']}, fp64 {w['fp64_gsps']} G spin-steps/s")
        wl[name] = w
        del phk
    out["workloads"] = wl
    return dictionary


def bench_mrf_match(K, ctx, torch, dictionary, no_cpu, n_pix=65536, reps=5):
    """Dictionary matching of a 256 x 256 fingerprint map against the
    simulated FISP dictionary: every pixel is a random entry times a random
    complex proton density plus 2 % complex Gaussian noise (seeded)."""
    n_e, n_t = dictionary.shape
    g = torch.Generator(device="cuda:0")
    g.manual_seed(4040)
    d = torch.from_numpy(np.stack([dictionary.real, dictionary.imag], -1)).to("cuda:0").contiguous()
    truth = torch.randint(0, n_e, (n_pix,), generator=g, device="cuda:0")
    amp = torch.rand(n_pix, generator=g, device="cuda:0") * 0.9 + 0.1
    ph = torch.rand(n_pix, generator=g, device="cuda:0") * 6.283185307179586
    dc = torch.view_as_complex(d)
    sigma = 0.02 * dc.abs().amax(dim=1)[truth]
    noise = torch.randn(n_pix, n_t, 2, generator=g, device="cuda:0") * (sigma / np.sqrt(2.0))[:, None, None]
    x = dc[truth] * (amp * torch.exp(1j * ph)).to(torch.complex64)[:, None]
    x = (torch.view_as_real(x) + noise).contiguous()
    best = torch.empty(n_pix, dtype=torch.int32, device="cuda:0")
    proj = torch.empty((n_pix, 2), dtype=torch.float64, device="cuda:0")
    ctx.mrf_match(d, x, where="device", best=best, proj=proj)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.mrf_match(d, x, where="device", best=best, proj=proj)
    torch.cuda.synchronize()
    t_call = (time.perf_counter() - t0) / reps
    st = ctx.kernel_stats("mrf")
    ctx.profile(False)
    k_ms = st["total_ms"] / max(st["launches"], 1)
    flop = 8.0 * n_pix * n_e * n_t
    achieved = flop / (k_ms * 1e-3) / 1e12
    b = best.cpu().numpy()
    traffic = load_stored("traffic_k_mrf_match.json", kernel_source_hash(("komahip_mrf.hip", "komahip_mrf.h")))
    out = {"pixels": n_pix, "entries": n_e, "trs": n_t, "call_ms": round(t_call * 1e3, 3),
           "kernel_ms": round(k_ms, 4), "flop_per_unit": 8,
           "unit_def": "one complex multiply-add of <d, x> (pixel x entry x TR)",
           "roofline": {"bound": "mfma", "kernel": "k_mrf_match (v_mfma_f32_32x32x16_f16, fused argmax)",
                        "achieved": round(achieved, 2), "peak": PEAK_FP16, "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_FP16, 4),
                        "traffic": traffic["bytes_per_launch"] if traffic else None,
                        "traffic_source": traffic["source"] if traffic else None},
           "recovered_fraction": float(np.mean(b == truth.cpu().numpy()))}
    if not no_cpu:  # against the FP64 definition on the caller's inputs, a seeded sample of pixels
        from oracle import mrf_match as M
        idx = np.sort(np.random.default_rng(4141).choice(n_pix, 512, replace=False))
        xs = x[idx].cpu().numpy()
        xs = (xs[..., 0] + 1j * xs[..., 1]).astype(np.complex64)
        t0 = time.perf_counter()
        j = M.judge_picks(b[idx], dictionary, xs)
        t_ref = time.perf_counter() - t0
        rr = M.match_rounded(dictionary, xs)[0]
        j["identical_to_binary16_argmax"] = int(np.sum(b[idx] == rr))
        out["parity_vs_definition"] = j
        out["cpu_reference_ms_per_pixel"] = round(t_ref / len(idx) * 1e3, 3)
    log(f"[bench] mrf match {n_pix} px x {n_e} entries x {n_t} TR: kernel {k_ms:.3f} ms, "
        f"{achieved:.1f} TFLOP/s, recovered {out['recovered_fraction']:.4f}; parity {out.get('parity_vs_definition')}")
    # rank-5 compression (the paper's LRTV dictionary rank), then matching in the
    # compressed domain
    rank = 5
    basis = torch.empty((n_t, rank, 2), dtype=torch.float64, device="cuda:0")
    sv = torch.empty(rank, dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    K._check(K.lib().koma_mrf_svd(ctx.h, K._ptr(d), n_e, n_t, rank, 11, 30, K.KOMA_DEVICE, None, K._ptr(basis),
                                  K._ptr(sv)), ctx.h)
    torch.cuda.synchronize()
    t_svd = time.perf_counter() - t0
    cd = torch.empty((n_e, rank, 2), dtype=torch.float32, device="cuda:0")
    cx = torch.empty((n_pix, rank, 2), dtype=torch.float32, device="cuda:0")
    t0 = time.perf_counter()
    for rows, n_rows, outp in ((d, n_e, cd), (x, n_pix, cx)):
        K._check(K.lib().koma_mrf_project(ctx.h, K._ptr(rows), n_rows, n_t, K._ptr(basis), rank, K.KOMA_DEVICE, None,
                                          K._ptr(outp)), ctx.h)
    bc = torch.empty_like(best)
    pc = torch.empty_like(proj)
    ctx.mrf_match(cd, cx, where="device", best=bc, proj=pc)
    torch.cuda.synchronize()
    t_lr = time.perf_counter() - t0
    bcn = bc.cpu().numpy()
    out["low_rank"] = {"rank": rank, "svd_ms": round(t_svd * 1e3, 2), "project_and_match_ms": round(t_lr * 1e3, 3),
                       "singular_values": [round(float(v), 4) for v in sv.cpu().numpy()],
                       "agreement_with_full": float(np.mean(bcn == b)),
                       "recovered_fraction": float(np.mean(bcn == truth.cpu().numpy()))}
    log(f"[bench] rank-{rank} compression: svd {t_svd * 1e3:.1f} ms, project + match {t_lr * 1e3:.2f} ms, "
        f"agreement with full matching {out['low_rank']['agreement_with_full']:.4f}")
    return out


def bench_extras(K, ctx, torch, W, out):
    # sequence-aware time stepping: the same sequences from their block
    # form, discretised by the library to the minimal grid
    seqaware = {}
    for k, blocks_fn in ((1, W.gre_blocks), (2, W.epi_blocks)):
        sck, phk, seqk = W.config(k)
        blocks = blocks_fn()
        t0 = time.perf_counter()
        m = K.koma_discretize(blocks)
        t_disc = time.perf_counter() - t0
        rep = 5 if k == 1 else 50
        tr, sr, _ = run_workload(K, ctx, torch, sck, phk, seqk, "mixed", rep, 1)
        tm, sm, _ = run_workload(K, ctx, torch, sck, phk, m, "mixed", rep, 1)
        name = W.WORKLOAD_NAMES[k].split(" ")[0]
        seqaware[name] = {
            "blocks": len(blocks), "raster_intervals": seqk.n_int, "minimal_intervals": m.n_int,
            "discretise_ms": round(t_disc * 1e3, 3),
            "raster_ms": round(tr * 1e3, 3), "minimal_ms": round(tm * 1e3, 3),
            "speedup": round(tr / tm, 3), "minimal_vs_raster": err(sm, sr)}
        log(f"[bench] minimal grid {name}: {m.n_int} vs {seqk.n_int} intervals, "
            f"{tm * 1e3:.3f} vs {tr * 1e3:.3f} ms")
    out["sequence_aware"] = seqaware
    # motion (the paper's u_y = v_y t, v_y = 0.1 m/s) and 8 receive coils on epi256
    sc, ph, seq = W.config(2)
    ext = {}
    for tag, phx in (("motion_vy0.1", W.with_velocity(ph, (0.0, 0.1, 0.0))), ("coils8", W.with_coils(ph, 8))):
        tx, _, _ = run_workload(K, ctx, torch, sc, phx, seq, "mixed", 5, 1)
        ext[tag] = {"ms": round(tx * 1e3, 3), "gsps": round(ph.n * seq.n_int / tx / 1e9, 3),
                    "signals": phx.n_coils or 1}
        log(f"[bench] epi256 {tag}: {tx * 1e3:.3f} ms")
    out["extensions"] = ext


PROFILE_WORKLOADS = {"gre64": 1, "epi256": 2, "mrf": 4, "seepi": 5}


def profile_workload(K, ctx, torch, W, args):
    """One workload only, for profiler runs (kernel traces, counters): the
    named workload's simulation in the chosen forms (``--steps`` pipelined
    steps after ``--warmup``), the MRF matching of a simulated dictionary
    (``mrf_match``: ``--steps`` calls), or a plain 1 GiB device copy
    (``copy``: the reference for scaling byte counters). Prints one JSON line
    of times; no oracle, no CPU baseline."""
    out = {"workload": args.workload, "steps": args.steps, "warmup": args.warmup}
    forms = [f for f in args.forms.split(",") if f]
    if args.workload == "copy":
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(max(args.steps, 1)):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_bytes_read"] = out["copy_bytes_written"] = a.numel() * 4
        return out
    if args.workload == "mrf_match":
        sc, ph, seq = W.config(4)
        _, s, _ = run_workload(K, ctx, torch, sc, ph, seq, "mixed", 1, 0)
        d = s.astype(np.complex64)
        n_pix = 65536
        rng = np.random.default_rng(4040)
        x = d[rng.integers(0, d.shape[0], n_pix)] * np.complex64(0.7 + 0.2j)
        x = x + (0.02 * rng.normal(size=x.shape) * np.abs(x).max()).astype(np.float32)
        dd = torch.from_numpy(np.stack([d.real, d.imag], -1)).to("cuda:0").contiguous()
        xd = torch.from_numpy(np.stack([x.real, x.imag], -1).astype(np.float32)).to("cuda:0").contiguous()
        best = torch.empty(n_pix, dtype=torch.int32, device="cuda:0")
        proj = torch.empty((n_pix, 2), dtype=torch.float64, device="cuda:0")
        for _ in range(args.warmup):
            ctx.mrf_match(dd, xd, where="device", best=best, proj=proj)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.mrf_match(dd, xd, where="device", best=best, proj=proj)
        torch.cuda.synchronize()
        out["call_ms"] = round((time.perf_counter() - t0) / max(args.steps, 1) * 1e3, 4)
        out.update(pixels=n_pix, entries=int(d.shape[0]), trs=int(d.shape[1]))
        return out
    sc, ph, seq = W.config(PROFILE_WORKLOADS[args.workload])
    out.update(spins=ph.n, intervals=seq.n_int, adc=seq.n_adc)
    for prec in forms:
        t, _, _ = run_workload(K, ctx, torch, sc, ph, seq, prec, args.steps, args.warmup, 0, True)
        out[f"{prec}_ms_per_step"] = round(t * 1e3, 4)
        log(f"[bench] {args.workload} {prec}: {t * 1e3:.3f} ms/step")
    return out


def gpu_clocks():
    """Shader clock levels of the GPU as the driver reports them (sysfs,
    read-only), to put box-to-box differences in context; None if absent."""
    import glob
    for f in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            lines = open(f).read().strip().splitlines()
        except OSError:
            continue
        if lines:
            return {"levels": [ln.strip() for ln in lines][:8], "source": f}
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed headline steps")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--epi-steps", type=int, default=200, help="timed steps of the epi256 workload")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline and oracle errors")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--serving-warmup", type=int, default=50)
    ap.add_argument("--cpu-spins", type=int, default=16384, help="oracle subset on every thread")
    ap.add_argument("--cpu-spins-1t", type=int, default=1024, help="oracle subset on one thread")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration runs)")
    ap.add_argument("--workload", choices=sorted(PROFILE_WORKLOADS) + ["mrf_match", "copy"], default=None,
                    help="run only this workload and print its times (for profiler runs)")
    ap.add_argument("--forms", default="mixed,fp64", help="precision forms of --workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: spins would shard across GPUs with one "
                                   "final signal sum, which is not implemented; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2301_02702_amd import komahip as K
    from paper_2301_02702_amd import workloads as W

    K.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    khash = kernel_source_hash()
    ctx = K.Context(0, "mixed")
    if args.workload:
        out = profile_workload(K, ctx, torch, W, args)
        out["kernel_hash"] = khash
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    out = bench_headline(K, ctx, torch, W, args, khash)
    out["kernel_hash"] = khash
    if not args.no_extra:
        dictionary = bench_secondary(K, ctx, torch, W, args, out)
        bench_extras(K, ctx, torch, W, out)
        out["mrf_match"] = bench_mrf_match(K, ctx, torch, dictionary, args.no_cpu)
    if not args.no_serving:
        from paper_2301_02702_amd import serve
        log(f"[bench] serving: {args.serving_requests} requests (+{args.serving_warmup} warm-up) ...")
        out["serving"] = serve.benchmark(ctx_device=0, n_requests=args.serving_requests,
                                         n_warm=args.serving_warmup, log=log)
    out["gpu_sclk"] = gpu_clocks()
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 2 * a.numel() * 4
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
