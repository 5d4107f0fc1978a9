"""Parity at the full workload sizes, in the launch configuration the
benchmark uses (default configuration, device-resident phantom).

* MRF batch (4e6 spins, 10,000 dictionary entries): every entry is an
  independent output the oracle can compute on its own, so a seeded sample of
  entries is compared one by one.
* Multi-slice SE-EPI (5e6 spins, 327,680 samples): one output needs every
  spin, so the check uses linearity, which holds at any size: the FP64 form on
  the full phantom minus the FP64 form on the phantom without a seeded subset
  S equals the oracle on S; the mixed form is compared with the FP64 form at
  full size.
"""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W
from tests._gpu import check, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2301_02702_amd import komahip
    komahip.lib()
    return komahip


def run_device(K, ctx, sc, ph, seq):
    import torch
    dph = K.device_phantom(ph)
    sig = torch.zeros((ph.n_groups, seq.n_adc, 2), dtype=torch.float64, device="cuda:0")
    ctx.simulate(sc, dph, seq, where="device", sig=sig)
    s = sig.cpu().numpy()
    return s[..., 0] + 1j * s[..., 1]


def test_mrf_full_batch_sampled_entries(K):
    import oracle
    sc, ph, seq = W.config(4)
    rng = np.random.default_rng(4004)
    entries = np.sort(rng.choice(ph.n_groups, 48, replace=False))
    ctx = K.Context(0, "mixed")
    try:
        ref = np.stack([oracle.simulate(sc, ph.groups(int(e), int(e) + 1), seq, mode=oracle.MODE_BLOCK)[0]
                        for e in entries])
        for prec in ("fp64", "mixed"):
            say(f"[full] mrf {prec}")
            ctx.set_config(prec)
            got = run_device(K, ctx, sc, ph, seq)
            # per entry: NRMSE and largest sample error, normalised by the entry's max|oracle|
            check(got[entries], ref, prec, f"full mrf, {len(entries)} sampled entries")
    finally:
        ctx.close()


def test_seepi_full_linearity_against_oracle_subset(K):
    import oracle
    sc, ph, seq = W.config(5)
    rng = np.random.default_rng(5005)
    idx = np.sort(rng.choice(ph.n, 2000, replace=False))
    keep = np.ones(ph.n, dtype=bool)
    keep[idx] = False
    rest = ph.subset(np.nonzero(keep)[0])
    ctx = K.Context(0, "fp64")
    try:
        say("[full] seepi fp64 full")
        full64 = run_device(K, ctx, sc, ph, seq)[0]
        say("[full] seepi fp64 without the subset")
        rest64 = run_device(K, ctx, sc, rest, seq)[0]
        ref = oracle.simulate(sc, ph.subset(idx), seq, mode=oracle.MODE_BLOCK)[0]
        # the difference cancels 2,500x in magnitude, so FP64 rounding of the
        # full sums (~1e-16 relative) shows at ~3e-13 here
        check(full64 - rest64, ref, "fp64", "full seepi, (full - rest) vs oracle(subset)")
        ctx.set_config("mixed")
        say("[full] seepi mixed full")
        mixed = run_device(K, ctx, sc, ph, seq)[0]
        check(mixed, full64, "mixed", "full seepi, mixed vs fp64 at full size")
    finally:
        ctx.close()
