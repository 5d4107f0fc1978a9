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

The paper does not fix a precision. The library takes the decision on
half-precision operands: every row (dictionary entry or fingerprint) is
scaled by an exact power of two so that its largest component magnitude
lies in [0.5, 1), and each real and imaginary part is rounded to the
nearest IEEE binary16 value (ties to even). ``match_rounded`` applies that
same rounding and then evaluates the definition in FP64; ``match`` is the
definition on the unrounded inputs.
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
