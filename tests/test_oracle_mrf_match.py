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
