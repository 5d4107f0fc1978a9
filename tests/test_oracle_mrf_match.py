"""Pins of the reference MRF dictionary matching (maximum normalised dot
product, the paper's Full-Dict matching in its MRF experiment)."""
import numpy as np
import pytest

from paper_2301_02702_amd import workloads as W


@pytest.fixture(scope="module")
def M():
    from oracle import mrf_match
    return mrf_match


def random_dict(rng, n_e, n_t):
    return (rng.normal(size=(n_e, n_t)) + 1j * rng.normal(size=(n_e, n_t))) * rng.uniform(0.1, 3.0, (n_e, 1))


def test_brute_force_loop(M):
    rng = np.random.default_rng(1)
    d = random_dict(rng, 7, 5)
    x = rng.normal(size=(4, 5)) + 1j * rng.normal(size=(4, 5))
    best, proj, score = M.match(d, x)
    for p in range(4):
        vals = []
        for e in range(7):
            nrm = sum(abs(v) ** 2 for v in d[e]) ** 0.5
            ip = sum(np.conj(d[e][t]) * x[p][t] for t in range(5))
            vals.append((abs(ip) / nrm, ip / nrm))
        e_best = max(range(7), key=lambda e: vals[e][0])
        assert best[p] == e_best
        assert abs(proj[p] - vals[e_best][1]) < 1e-12
        assert abs(score[p] - vals[e_best][0] ** 2) < 1e-12 * score[p]


def test_noise_free_fingerprints_recover_entry_and_scale(M):
    rng = np.random.default_rng(2)
    d = random_dict(rng, 50, 64)
    e = rng.integers(0, 50, 30)
    c = rng.normal(size=30) + 1j * rng.normal(size=30)
    x = c[:, None] * d[e]
    best, proj, score = M.match(d, x)
    nrm = np.linalg.norm(d[e], axis=1)
    assert np.array_equal(best, e)
    assert np.allclose(proj, c * nrm, rtol=1e-12)
    # Cauchy-Schwarz: the score is |x|^2 exactly for a noise-free fingerprint
    assert np.allclose(score, np.linalg.norm(x, axis=1) ** 2, rtol=1e-12)
    xn = x + 0.3 * (rng.normal(size=x.shape) + 1j * rng.normal(size=x.shape))
    _, _, s2 = M.match(d, xn)
    assert np.all(s2 <= np.linalg.norm(xn, axis=1) ** 2 * (1 + 1e-12))


def test_scale_invariance(M):
    rng = np.random.default_rng(3)
    d = random_dict(rng, 40, 32)
    x = rng.normal(size=(10, 32)) + 1j * rng.normal(size=(10, 32))
    b1, p1, _ = M.match(d, x)
    alpha = 2.5 * np.exp(0.7j)
    b2, p2, _ = M.match(d * 3.0, x * alpha)
    assert np.array_equal(b1, b2)
    assert np.allclose(p2, alpha * p1, rtol=1e-12)


def test_half_rounding_of_rows(M):
    rng = np.random.default_rng(4)
    a = (random_dict(rng, 20, 16) * np.logspace(-6, 6, 20)[:, None]).astype(np.complex64)
    h, k = M.round_rows_half(a)
    scaled = a.astype(np.complex128) * np.ldexp(1.0, k)[:, None]
    mx = np.maximum(np.abs(scaled.real).max(1), np.abs(scaled.imag).max(1))
    assert np.all((mx >= 0.5) & (mx < 1.0))
    # every rounded part is a binary16 value within half an ulp of the scaled one
    for part, ref in ((h.real, scaled.real), (h.imag, scaled.imag)):
        assert np.array_equal(part, part.astype(np.float16).astype(np.float64))
        ulp = np.spacing(np.abs(ref).astype(np.float16)).astype(np.float64)
        assert np.all(np.abs(part - ref) <= 0.5 * ulp + 1e-300)


def test_rounded_matching_agrees_on_separated_entries(M):
    rng = np.random.default_rng(5)
    d = random_dict(rng, 64, 100).astype(np.complex64)
    e = rng.integers(0, 64, 40)
    x = (d[e] * (1 + 0.5j) + 0.05 * (rng.normal(size=(40, 100)) + 1j * rng.normal(size=(40, 100)))).astype(np.complex64)
    b, p, _ = M.match(d, x)
    br, pr, _, _ = M.match_rounded(d, x)
    assert np.array_equal(b, e) and np.array_equal(br, e)
    assert np.allclose(pr, p, rtol=2e-3)


def test_simulated_mrf_dictionary_identifies_t1_t2(M, oracle_mod):
    """A small FISP dictionary simulated by the oracle (6 x 6 T1/T2 grid,
    40 isochromats per entry, 300 TRs): noisy copies of entries are matched
    back to their own T1/T2."""
    seq = W.mrf_sequence(n_tr=300)
    ph = W.mrf_phantom(n_t1=6, n_t2=6, n_iso=40)
    dic = oracle_mod.simulate(W.Scanner(), ph, seq, mode=oracle_mod.MODE_BLOCK)
    rng = np.random.default_rng(6)
    e = rng.integers(0, 36, 25)
    sig = np.abs(dic[e]).max(axis=1, keepdims=True)
    x = dic[e] * 0.8 + 0.01 * sig * (rng.normal(size=(25, 300)) + 1j * rng.normal(size=(25, 300)))
    best, proj, _ = M.match(dic, x)
    assert np.array_equal(best, e)
    assert np.allclose(np.abs(proj), 0.8 * np.linalg.norm(dic[e], axis=1), rtol=0.02)


def test_svd_basis_recovers_a_planted_subspace(M):
    """A dictionary built as A B with B (rank x n_t) of orthonormal rows and
    A with orthogonal columns of known norms: the leading right singular
    vectors span B's rows and the singular values are those norms."""
    rng = np.random.default_rng(11)
    n_e, n_t, r = 300, 80, 5
    q, _ = np.linalg.qr(rng.normal(size=(n_t, r)) + 1j * rng.normal(size=(n_t, r)))
    b = q.conj().T                                   # r x n_t, orthonormal rows
    qa, _ = np.linalg.qr(rng.normal(size=(n_e, r)) + 1j * rng.normal(size=(n_e, r)))
    norms = np.array([50.0, 20.0, 7.0, 3.0, 1.0])
    d = (qa * norms) @ b
    v, s = M.svd_basis(d, r)
    assert np.allclose(s, norms, rtol=1e-12)
    pv = v @ v.conj().T
    pb = b.conj().T @ b
    assert np.max(np.abs(pv - pb)) < 1e-12
    assert np.allclose(v.conj().T @ v, np.eye(r), atol=1e-12)


def test_projection_preserves_inner_products_in_the_span(M):
    rng = np.random.default_rng(12)
    q, _ = np.linalg.qr(rng.normal(size=(60, 4)) + 1j * rng.normal(size=(60, 4)))
    coef = rng.normal(size=(10, 4)) + 1j * rng.normal(size=(10, 4))
    rows = coef @ q.conj().T                          # in span(q)
    c = M.project(rows, q)
    assert np.allclose(c, coef, atol=1e-12)
    assert np.allclose(rows @ rows.conj().T, c @ c.conj().T, atol=1e-12)


def _emulated_library_cosines(d, x):
    """Brute-force emulation of a half-precision decision: rows scaled by a
    power of two and rounded to binary16 (numpy's own float16 conversion),
    products formed exactly and summed one by one in float32, the entry's
    squared norm summed the same way; cosine against the exact ||x||."""
    def half_rows(a):
        a = np.asarray(a, dtype=np.complex64)
        out = []
        for row in a:
            m = max(np.max(np.abs(row.real)), np.max(np.abs(row.imag)))
            k = -np.frexp(m)[1] if m > 0 else 0
            s = np.float32(2.0 ** k)
            out.append(((row.real * s).astype(np.float16), (row.imag * s).astype(np.float16), k))
        return out
    dh, xh = half_rows(d), half_rows(x)
    nx = np.linalg.norm(np.asarray(x, dtype=np.complex128), axis=1)
    c = np.zeros((len(xh), len(dh)))
    for p, (xr, xi, kx) in enumerate(xh):
        for e, (dr, di, kd) in enumerate(dh):
            re = np.float32(0)
            im = np.float32(0)
            n2 = np.float32(0)
            for t in range(len(dr)):
                a, b = np.float32(dr[t]), np.float32(di[t])
                u, v = np.float32(xr[t]), np.float32(xi[t])
                re = np.float32(np.float32(re + a * u) + b * v)
                im = np.float32(np.float32(im + a * v) - b * u)
                n2 = np.float32(np.float32(n2 + a * a) + b * b)
            if n2 > 0 and nx[p] > 0:
                # back to the caller's units: x' carries 2^kx
                c[p, e] = np.sqrt(float(re) ** 2 + float(im) ** 2) * 2.0 ** -kx / (np.sqrt(float(n2)) * nx[p])
    return c


@pytest.mark.parametrize("seed,n_t,tiny", [(0, 40, False), (1, 300, False), (2, 64, True)])
def test_decision_bound_covers_an_emulated_half_precision_decision(M, seed, n_t, tiny):
    """decision_bound against brute force: every emulated binary16/FP32
    cosine lies within beta of the FP64 cosine of the unrounded inputs
    (including rows whose small components fall into binary16's subnormal
    range); and judge_picks accepts the emulated argmax while rejecting a
    pick that is clearly worse."""
    rng = np.random.default_rng(300 + seed)
    d = random_dict(rng, 12, n_t).astype(np.complex64)
    if tiny:  # components spanning 1e-9 .. 1 of the row maximum
        d = (d * np.exp(rng.uniform(-20, 0, d.shape))).astype(np.complex64)
    e = rng.integers(0, 12, 9)
    x = (d[e] * (0.3 - 0.6j) + 0.2 * random_dict(rng, 9, n_t)).astype(np.complex64)
    c = M.cosines(d, x)
    ce = _emulated_library_cosines(d, x)
    beta = M.decision_bound(n_t)
    gap = float(np.max(np.abs(ce - c)))
    assert gap <= beta, (gap, beta)
    assert gap > 1e-7  # the emulation really rounds
    j = M.judge_picks(np.argmax(ce, axis=1), d, x)
    assert j["valid"]
    worst = np.argmin(c, axis=1)
    assert not M.judge_picks(worst, d, x)["valid"]


def test_cosines_are_the_definition(M):
    """argmax of the cosines is the definition's pick; a noise-free scaled
    copy has cosine 1; Cauchy-Schwarz bounds every cosine by 1."""
    rng = np.random.default_rng(12)
    d = random_dict(rng, 20, 30)
    x = np.concatenate([d[[3, 7]] * (2 - 1j), random_dict(rng, 5, 30)])
    c = M.cosines(d, x)
    best, _, score = M.match(d, x)
    assert np.array_equal(np.argmax(c, axis=1), best)
    assert abs(c[0, 3] - 1) < 1e-14 and abs(c[1, 7] - 1) < 1e-14
    assert np.all(c <= 1 + 1e-14)
    nx2 = np.sum(np.abs(x) ** 2, axis=1)
    assert np.allclose(c[np.arange(len(x)), best] ** 2 * nx2, score, rtol=1e-12)
