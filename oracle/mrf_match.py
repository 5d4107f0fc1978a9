"""Plain reference of MR-fingerprinting dictionary matching.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU-baseline leg
use it; the product never imports it, and it shares no code with the
library.

Section "MR Fingerprinting" (the paper's MRF experiment, Full-Dict
reconstruction): each pixel's fingerprint x (one complex value per TR) is
assigned the dictionary entry with the maximum dot product, the entries
being normalised: best(x) = argmax_e |<d_e, x>| / ||d_e||, with
<d, x> = sum_t conj(d_t) x_t. The projection <d_best, x> / ||d_best|| is
the pixel's complex proton-density scale (relative to the entry's own
scale).

The paper does not fix a precision. ``match`` is the definition on the
caller's inputs in FP64, and ``judge_picks`` checks a pick against it with
the error bound of ``decision_bound``. The library takes the decision on
half-precision operands: every row (dictionary entry or fingerprint) is
scaled by an exact power of two so that its largest component magnitude
lies in [0.5, 1), and each real and imaginary part is rounded to the
nearest IEEE binary16 value (ties to even). ``match_rounded`` applies that
same rounding and then evaluates the definition in FP64 (a diagnostic of
where a pick differs from the definition, not the parity reference).
"""
from __future__ import annotations

import numpy as np


def match(dictionary, x):
    """FP64 maximum normalised dot product. Returns (best [n_p] int64,
    projection [n_p] complex128, score [n_p] float64 = |<d_best, x>|^2 / ||d_best||^2)."""
    d = np.asarray(dictionary, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128)
    norm2 = np.sum(np.abs(d) ** 2, axis=1)
    ip = x @ d.conj().T                       # <d_e, x> for every pixel and entry
    score = np.abs(ip) ** 2 / np.where(norm2 > 0, norm2, np.inf)[None, :]
    best = np.argmax(score, axis=1)           # ties: the lowest index
    rows = np.arange(x.shape[0])
    proj = ip[rows, best] / np.sqrt(norm2[best])
    return best.astype(np.int64), proj, score[rows, best]


def cosines(dictionary, x):
    """FP64 |<d_e, x>| / (||d_e|| ||x||) for every pixel and entry [n_p, n_e]
    (0 where either row is zero): the definition's score, normalised so that
    it lies in [0, 1] and its argmax over e is the definition's pick."""
    d = np.asarray(dictionary, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128)
    nd = np.sqrt(np.sum(np.abs(d) ** 2, axis=1))
    nx = np.sqrt(np.sum(np.abs(x) ** 2, axis=1))
    ip = np.abs(x @ d.conj().T)
    den = nx[:, None] * nd[None, :]
    return np.where(den > 0, ip / np.where(den > 0, den, 1.0), 0.0)


def decision_bound(n_t):
    """Bound beta on |c'_e - c_e| for every entry e, where c_e is the FP64
    cosine of the unrounded inputs and c'_e the cosine the library ranks by
    (binary16 rows, FP32 accumulation of exact products, FP32 norm).

    * Rounding a row to binary16 after the exact power-of-two scaling (largest
      |Re|, |Im| in [0.5, 1), so ||row|| >= 0.5): each normal component moves
      by at most u16 = 2^-11 of itself, each subnormal one by at most 2^-25,
      so ||delta row|| <= eps ||row|| with eps = u16 + 2^-24 sqrt(2 n_t).
    * |<d', x'> - <d, x>| <= (2 eps + eps^2) ||d|| ||x|| (Cauchy-Schwarz).
    * Re and Im of <d', x'> are sums of 2 n_t exact products in FP32: error
      <= gamma ||d'|| ||x'|| each, gamma = m u32 / (1 - m u32), m = 2 n_t,
      u32 = 2^-24; sqrt(2) gamma for the modulus.
    * ||d'|| is within eps of ||d||, and its FP32 square within gamma.
    * A few FP32 roundings of the score itself (|.|^2, 1/||d'||^2, product).
    To first order beta = 3 eps + (sqrt(2) + 1/2) gamma; the value returned
    rounds the constants up. If c_best - c_second > 2 beta the library must
    pick the definition's entry; otherwise its pick must have c >= c_best -
    2 beta."""
    u16 = 2.0 ** -11
    u32 = 2.0 ** -24
    eps = u16 + u32 * np.sqrt(2.0 * n_t)
    gam = 2.0 * n_t * u32 / (1.0 - 2.0 * n_t * u32)
    return 3.0 * eps + 3.0 * eps ** 2 + 2.0 * gam + 4.0 * u32


def judge_picks(best, dictionary, x):
    """The library's picks `best` against the definition. Returns a dict:
    identical (picks equal to the FP64 argmax), clear (pixels whose best and
    second-best cosines differ by more than 2 beta), clear_identical,
    valid (every pick within 2 beta of the best cosine, and identical where
    the gap is clear), worst_shortfall (largest c_best - c_pick)."""
    c = cosines(dictionary, x)
    n_p, n_e = c.shape
    rows = np.arange(n_p)
    ref = np.argmax(c, axis=1)
    cb = c[rows, ref]
    if n_e > 1:
        second = np.partition(c, n_e - 2, axis=1)[:, n_e - 2]
    else:
        second = np.full(n_p, -np.inf)
    beta = decision_bound(np.shape(dictionary)[1])
    clear = (cb - second) > 2.0 * beta
    best = np.asarray(best)
    same = best == ref
    short = cb - c[rows, best]
    valid = bool(np.all(same[clear]) and np.all(short <= 2.0 * beta))
    return {"pixels": int(n_p), "identical": int(np.sum(same)), "clear": int(np.sum(clear)),
            "clear_identical": int(np.sum(same & clear)), "valid": valid,
            "worst_shortfall": float(np.max(short)) if n_p else 0.0, "bound_2beta": float(2.0 * beta)}


def round_rows_half(a):
    """Scale every row by 2^k (exact) so that its largest |Re| or |Im| is in
    [0.5, 1), round real and imaginary parts to binary16; return the rounded
    values (as complex128, in the scaled units) and k per row."""
    a = np.asarray(a, dtype=np.complex64)
    m = np.maximum(np.max(np.abs(a.real), axis=1), np.max(np.abs(a.imag), axis=1)).astype(np.float64)
    _, e = np.frexp(np.where(m > 0, m, 1.0))  # m = f 2^e, f in [0.5, 1)
    k = -e
    s = np.ldexp(np.ones_like(m), k)[:, None]
    re = (a.real.astype(np.float64) * s).astype(np.float16).astype(np.float64)
    im = (a.imag.astype(np.float64) * s).astype(np.float16).astype(np.float64)
    return re + 1j * im, k


def match_rounded(dictionary, x):
    """The definition evaluated in FP64 on the half-precision operands the
    library uses. Returns (best, projection in the caller's units, score of
    the rounded operands, all scores [n_p, n_e])."""
    dh, kd = round_rows_half(dictionary)
    xh, kx = round_rows_half(x)
    norm2 = np.sum(np.abs(dh) ** 2, axis=1)
    ip = xh @ dh.conj().T
    score = np.abs(ip) ** 2 / np.where(norm2 > 0, norm2, np.inf)[None, :]
    best = np.argmax(score, axis=1)
    rows = np.arange(xh.shape[0])
    # back to the caller's units: <d/||d||, x> is invariant to d's scale and
    # scales as 2^-kx with x's
    proj = ip[rows, best] / np.sqrt(norm2[best]) * np.ldexp(1.0, -kx)
    return best.astype(np.int64), proj, score[rows, best], score


def svd_basis(dictionary, rank):
    """The `rank` leading right singular vectors (columns of V, [n_t, rank])
    and singular values of the dictionary, D = U S V^H, in FP64 (the low-rank
    compression of the paper's LRTV matching, rank 5)."""
    d = np.asarray(dictionary, dtype=np.complex128)
    _, s, vh = np.linalg.svd(d, full_matrices=False)
    return vh[:rank].conj().T, s[:rank]


def project(rows, basis):
    """Coefficients of rows in a basis: c_j = sum_t x_t basis[t, j]."""
    return np.asarray(rows, dtype=np.complex128) @ np.asarray(basis, dtype=np.complex128)
