"""GPU parity of MRF dictionary matching (MFMA contraction + fused argmax)
against the definition: the maximum normalised dot product in FP64 on the
caller's FP32 dictionary and fingerprints (oracle/mrf_match.py, ``match``).

The library takes the argmax on binary16 rows with FP32 accumulation, so
its cosine of each entry lies within beta (``decision_bound``, derived in
its docstring) of the definition's. Where the definition's best and
second-best cosines are more than 2 beta apart the picks must be identical;
elsewhere the library's pick must have a cosine within 2 beta of the best.
The projection <d, x>/||d|| of identical picks must agree within the same
rounding (3.1 eps ||x||). ``match_rounded`` (the definition on the
library's own binary16 operands) is printed as a diagnostic only.
"""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W
from tests._gpu import say

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


def check(best, proj, d, x, tag):
    from oracle import mrf_match as M
    j = M.judge_picks(best, d, x)
    rb, rp, _ = M.match(d, x)
    rr = M.match_rounded(d, x)[0]
    say(f"[mrf match] {tag}: {j['identical']}/{j['pixels']} picks equal to the definition's, "
        f"{j['clear_identical']}/{j['clear']} where the gap exceeds 2 beta = {j['bound_2beta']:.2e}; "
        f"worst cosine shortfall {j['worst_shortfall']:.2e}; "
        f"{int(np.sum(best == rr))} equal to the argmax on the library's binary16 operands")
    assert j["valid"], (tag, j)
    same = best == rb
    eps = 2.0 ** -11 + 2.0 ** -24 * np.sqrt(2.0 * d.shape[1])
    nx = np.linalg.norm(np.asarray(x, dtype=np.complex128), axis=1)
    assert np.all(np.abs(proj[same] - rp[same]) <= 3.1 * eps * nx[same] + 1e-300), tag


def rnd(rng, shape):
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex64)


@pytest.mark.parametrize("n_e,n_p,n_t", [(300, 500, 100), (64, 128, 8), (1, 7, 3), (257, 129, 1), (130, 300, 333)])
def test_random_operands_match_reference(ctx, n_e, n_p, n_t):
    """Ragged sizes over several tiles: entry and pixel tiles of 128,
    contraction slices of 16 TR values."""
    rng = np.random.default_rng(n_e * 7 + n_p + n_t)
    d = rnd(rng, (n_e, n_t)) * rng.uniform(0.01, 100.0, (n_e, 1)).astype(np.float32)
    e = rng.integers(0, n_e, n_p)
    x = (d[e] * (0.5 - 0.8j) + 0.3 * np.abs(d[e]).mean(1, keepdims=True) * rnd(rng, (n_p, n_t))).astype(np.complex64)
    best, proj = ctx.mrf_match(d, x)
    check(best, proj, d, x, f"random {n_e}x{n_p}x{n_t}")


def test_noise_free_fingerprints_pick_their_entry(ctx):
    """Fingerprints that are scaled copies of distinct random entries: the
    MFMA operand layout must put every product where it belongs."""
    rng = np.random.default_rng(7)
    d = rnd(rng, (1000, 200))
    e = rng.permutation(1000)[:640]
    c = (rng.uniform(0.1, 10, 640) * np.exp(1j * rng.uniform(0, 6.28, 640))).astype(np.complex64)
    x = (c[:, None] * d[e]).astype(np.complex64)
    best, proj = ctx.mrf_match(d, x)
    assert np.array_equal(best, e)
    nrm = np.linalg.norm(d[e].astype(np.complex128), axis=1)
    assert np.allclose(proj, c * nrm, rtol=2e-3)


def test_zero_rows(ctx):
    rng = np.random.default_rng(8)
    d = rnd(rng, (70, 16))
    d[3] = 0
    x = rnd(rng, (5, 16))
    x[2] = 0
    x[4] = d[3]  # zero
    best, proj = ctx.mrf_match(d, x)
    assert 3 not in set(best[[0, 1, 3]].tolist())
    assert best[2] == 0 and best[4] == 0 and proj[2] == 0 and proj[4] == 0  # all scores 0: lowest index


def test_device_path_is_the_host_path(ctx):
    import torch
    rng = np.random.default_rng(9)
    d = rnd(rng, (200, 50))
    x = rnd(rng, (333, 50))
    b1, p1 = ctx.mrf_match(d, x)
    td = torch.from_numpy(np.stack([d.real, d.imag], -1).astype(np.float32)).cuda()
    tx = torch.from_numpy(np.stack([x.real, x.imag], -1).astype(np.float32)).cuda()
    bb = torch.empty(333, dtype=torch.int32, device="cuda")
    pp = torch.empty((333, 2), dtype=torch.float64, device="cuda")
    ctx.mrf_match(td, tx, where="device", best=bb, proj=pp)
    p2 = pp.cpu().numpy()
    assert np.array_equal(b1, bb.cpu().numpy()) and np.array_equal(p1, p2[:, 0] + 1j * p2[:, 1])


def test_simulated_dictionary_recovers_t1_t2(ctx):
    """A FISP dictionary simulated on the GPU (40 T1/T2 entries, 1000 TRs):
    noisy scaled copies are matched back to their entries."""
    from tests._gpu import case
    sc, ph, seq = case("mrf40")
    ctx.set_config("mixed")
    dic = ctx.simulate(sc, ph, seq).astype(np.complex64)
    rng = np.random.default_rng(10)
    e = rng.integers(0, 40, 500)
    amp = np.abs(dic[e]).max(1, keepdims=True)
    x = (dic[e] * 0.7 + 0.01 * amp * rnd(rng, (500, seq.n_adc))).astype(np.complex64)
    best, proj = ctx.mrf_match(dic, x)
    check(best, proj, dic, x, "simulated mrf40")
    assert np.mean(best == e) > 0.99


def test_svd_recovers_a_planted_subspace(ctx):
    rng = np.random.default_rng(11)
    n_e, n_t, r = 3000, 200, 5
    q, _ = np.linalg.qr(rng.normal(size=(n_t, r)) + 1j * rng.normal(size=(n_t, r)))
    qa, _ = np.linalg.qr(rng.normal(size=(n_e, r)) + 1j * rng.normal(size=(n_e, r)))
    norms = np.array([50.0, 20.0, 7.0, 3.0, 1.0])
    d = ((qa * norms) @ q.conj().T).astype(np.complex64)
    v, s = ctx.mrf_svd(d, rank=r, oversample=3, iters=20)
    from oracle import mrf_match as M
    vr, sr = M.svd_basis(d, r)  # of the float32-rounded dictionary
    ep = np.max(np.abs(v @ v.conj().T - vr @ vr.conj().T))
    es = np.max(np.abs(s - sr) / sr)
    say(f"[mrf svd] planted rank {r}: projector diff {ep:.2e}, singular values rel {es:.2e}")
    assert ep < 1e-9 and es < 1e-9
    assert np.allclose(v.conj().T @ v, np.eye(r), atol=1e-10)


def test_svd_and_compressed_matching_of_a_simulated_dictionary(ctx):
    """The rank-5 basis of a GPU-simulated FISP dictionary against the FP64
    SVD, projection against the reference, and matching in the compressed
    domain against full matching."""
    from oracle import mrf_match as M
    from tests._gpu import case
    sc, ph, seq = case("mrf40")
    ctx.set_config("mixed")
    dic = ctx.simulate(sc, ph, seq).astype(np.complex64)
    v, s = ctx.mrf_svd(dic, rank=5)
    vr, sr = M.svd_basis(dic, 5)
    ep = np.max(np.abs(v @ v.conj().T - vr @ vr.conj().T))
    es = np.max(np.abs(s - sr) / sr)
    assert ep < 1e-6 and es < 1e-8, (ep, es)
    rng = np.random.default_rng(13)
    e = rng.integers(0, 40, 300)
    x = (dic[e] * 0.9 + 0.005 * np.abs(dic).max() * rnd(rng, (300, seq.n_adc))).astype(np.complex64)
    cd = ctx.mrf_project(dic, v)
    cx = ctx.mrf_project(x, v)
    assert np.allclose(cd, M.project(dic, v), rtol=1e-5, atol=1e-6 * np.abs(cd).max())
    bf, _ = ctx.mrf_match(dic, x)
    bc, _ = ctx.mrf_match(cd, cx)
    agree = float(np.mean(bf == bc))
    say(f"[mrf svd] mrf40 rank 5: projector diff {ep:.2e}, sv rel {es:.2e}, compressed vs full picks {agree:.3f}")
    assert agree > 0.95
