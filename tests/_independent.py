"""Independent numpy references used to pin the oracle.

None of this code follows the oracle's formulas: rotations are built from the
Rodrigues axis-angle matrix (not the spinor of Eq. Rot_exc), relaxation and
whole-interval solutions from the exact matrix exponential of the linear
Bloch system, k-space from an FFT, and the FISP train from an extended phase
graph (EPG) written from the Fourier-series picture of a voxel.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def rodrigues(axis, angle):
    """Right-handed rotation matrix by ``angle`` about the unit ``axis``."""
    n = np.asarray(axis, dtype=np.float64)
    n = n / np.linalg.norm(n)
    K = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def field_rotation(gamma, B, dt):
    """Solution operator of dM/dt = gamma M x B (constant B) over dt: a
    rotation about B by -gamma |B| dt."""
    nb = np.linalg.norm(B)
    if nb == 0.0:
        return np.eye(3)
    return rodrigues(B / nb, -gamma * nb * dt)


def relax_affine(dt, t1, t2, m0):
    """Exact solution of the relaxation ODE over dt as (A, b): M -> A M + b."""
    e1 = np.exp(-dt / t1)
    e2 = np.exp(-dt / t2)
    return np.diag([e2, e2, e1]), np.array([0.0, 0.0, m0 * (1 - e1)])


def bloch_generator(gamma, B, t1, t2, m0):
    """4x4 generator H with d/dt [M; 1] = H [M; 1] for the full Bloch
    equation with constant field B (paper's Eq. Bloch)."""
    bx, by, bz = B
    r1 = 0.0 if np.isinf(t1) else 1.0 / t1
    r2 = 0.0 if np.isinf(t2) else 1.0 / t2
    H = np.zeros((4, 4))
    H[:3, :3] = gamma * np.array([[0, bz, -by], [-bz, 0, bx], [by, -bx, 0]])
    H[0, 0] -= r2
    H[1, 1] -= r2
    H[2, 2] -= r1
    H[2, 3] = m0 * r1
    return H


def exact_interval(gamma, B, t1, t2, m0, dt, M):
    """Exact Bloch solution over dt with constant B (expm)."""
    v = expm(bloch_generator(gamma, B, t1, t2, m0) * dt) @ np.append(M, 1.0)
    return v[:3]


def brute_force(gamma, phantom, seq):
    """Per-interval rotation (Rodrigues about the full field, G taken as the
    interval mean) followed by the exact relaxation, for every spin; returns
    (signal [n_groups, n_adc], final M [n, 3]). Small inputs only."""
    n = phantom.n
    n_int = seq.n_int
    adc = set(int(k) for k in seq.adc_idx)
    adc_pos = {int(k): i for i, k in enumerate(seq.adc_idx)}
    goff = phantom.group_off if phantom.group_off is not None else np.array([0, n])
    sig = np.zeros((len(goff) - 1, seq.n_adc), dtype=np.complex128)
    M_all = np.zeros((n, 3))
    for j in range(n):
        g = int(np.searchsorted(goff, j, side="right") - 1)
        x = np.array([phantom.x[j], phantom.y[j], phantom.z[j]], dtype=np.float64)
        m0, t1, t2, dw = (float(phantom.pd[j]), float(phantom.t1[j]), float(phantom.t2[j]),
                          float(phantom.dw[j]))
        M = np.array([0.0, 0.0, m0])
        if 0 in adc:
            sig[g, adc_pos[0]] += M[0] + 1j * M[1]
        for i in range(n_int):
            dt = seq.t[i + 1] - seq.t[i]
            G = 0.5 * np.array([seq.gx[i] + seq.gx[i + 1], seq.gy[i] + seq.gy[i + 1],
                                seq.gz[i] + seq.gz[i + 1]])
            B = np.array([seq.b1[i].real, seq.b1[i].imag, x @ G + dw / gamma])
            M = field_rotation(gamma, B, dt) @ M
            A, b = relax_affine(dt, t1, t2, m0)
            M = A @ M + b
            if i + 1 in adc:
                sig[g, adc_pos[i + 1]] += M[0] + 1j * M[1]
        M_all[j] = M
    return sig, M_all


def rotation_to_transverse_coeffs(R):
    """Write M' = R M in the (Mxy, conj Mxy, Mz) basis:
    Mxy' = a Mxy + b conj(Mxy) + c Mz,  Mz' = Re(d Mxy) + e Mz."""
    a = 0.5 * (R[0, 0] + R[1, 1] + 1j * (R[1, 0] - R[0, 1]))
    b = 0.5 * (R[0, 0] - R[1, 1] + 1j * (R[1, 0] + R[0, 1]))
    c = R[0, 2] + 1j * R[1, 2]
    d = R[2, 0] - 1j * R[2, 1]
    e = R[2, 2]
    return a, b, c, d, e


def epg_voxel_mean(gamma, seq, t1, t2, m0, voxel, kmax=1100):
    """Extended phase graph of a voxel of length ``voxel`` along x for a
    sequence whose gradient moments between RF/ADC events are whole cycles
    across the voxel and whose RF acts while G = 0 and dw = 0.

    Mxy(x) = sum_k F[k] e^{i 2 pi k x / L}, Mz(x) = sum_k Z[k] e^{i 2 pi k x / L}.
    A uniform RF rotation mixes F[k], conj(F[-k]) and Z[k]; relaxation scales
    the states and regrows Z[0]; a gradient moment of one cycle per voxel
    (phase -2 pi x / L) moves F[k] to F[k-1]. Returns F[0] at every ADC point.
    """
    gbar = gamma / (2 * np.pi)
    K = kmax
    F = np.zeros(2 * K + 1, dtype=np.complex128)
    Z = np.zeros(2 * K + 1, dtype=np.complex128)
    Z[K] = m0
    adc = {int(k): i for i, k in enumerate(seq.adc_idx)}
    out = np.zeros(seq.n_adc, dtype=np.complex128)
    cycles = 0.0
    if 0 in adc:
        out[adc[0]] = F[K]
    for i in range(seq.n_int):
        dt = seq.t[i + 1] - seq.t[i]
        gm = 0.5 * (seq.gx[i] + seq.gx[i + 1])
        if seq.gy[i] or seq.gy[i + 1] or seq.gz[i] or seq.gz[i + 1]:
            raise ValueError("EPG reference supports Gx only")
        b1 = seq.b1[i]
        if b1 != 0:
            if gm != 0.0 or abs(cycles - round(cycles)) > 1e-9:
                raise ValueError("RF while dephased by a non-integer moment")
            R = field_rotation(gamma, np.array([b1.real, b1.imag, 0.0]), dt)
            a, b, c, d, e = rotation_to_transverse_coeffs(R)
            Fm = np.conj(F[::-1])  # conj(F[-k])
            F, Z = a * F + b * Fm + c * Z, 0.5 * (d * F + np.conj(d) * Fm) + e * Z
        else:
            cycles += gbar * gm * dt * voxel
        e1 = np.exp(-dt / t1)
        e2 = np.exp(-dt / t2)
        F = F * e2
        Z = Z * e1
        Z[K] += m0 * (1 - e1)
        c_round = round(cycles)
        if abs(cycles - c_round) < 1e-9 and c_round != 0:
            # whole cycles of dephasing: shift the transverse states
            s = int(c_round)
            F = np.roll(F, -s)
            if s > 0:
                F[-s:] = 0
            else:
                F[:-s] = 0
            cycles -= c_round
        if i + 1 in adc:
            if abs(cycles) > 1e-9:
                raise ValueError("ADC while dephased by a non-integer moment")
            out[adc[i + 1]] = F[K]
    return out
