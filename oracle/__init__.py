"""Python binding of the plain FP64 CPU oracle (``bloch_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it. The product library never loads or calls it, and
it shares no code with the GPU path. See ``bloch_oracle.c`` for what it
computes and which passage of the paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bloch_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MODE_STEP = 0   # splitting on every interval
MODE_BLOCK = 1  # precession blocks integrated (exact for piecewise-linear G)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                        "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_simulate.restype = ctypes.c_int
        lib.oracle_simulate.argtypes = [ctypes.c_double, i64] + [P] * 10 + [i64, P, P] + [i64, P, i64] + \
            [P] * 6 + [i64, P, ctypes.c_int, ctypes.c_int, P, P]
        lib.oracle_excite_step.restype = None
        lib.oracle_excite_step.argtypes = [ctypes.c_double, P, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, P]
        lib.oracle_relax_step.restype = None
        lib.oracle_relax_step.argtypes = [ctypes.c_double] * 4 + [P, P]
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def simulate(scanner, phantom, seq, mode: int = MODE_STEP, threads: int | None = None,
             want_m: bool = False):
    """Signal ``[n_groups, n_adc]`` complex128, or ``[n_coils, n_groups, n_adc]``
    when the phantom carries coil sensitivities (and ``[n, 3]`` final M if
    asked). A phantom with velocities ``vx, vy, vz`` moves as x + v t."""
    lib = _load()
    n = phantom.n
    ng = phantom.n_groups
    sens = getattr(phantom, "sens", None)
    nc = 0 if sens is None else int(sens.shape[0])
    sig = np.zeros((max(nc, 1), ng, seq.n_adc, 2), dtype=np.float64)
    m = np.zeros((n, 3), dtype=np.float64) if want_m else None
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)  # noqa: E731
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
    arrs = [f32(getattr(phantom, k)) for k in ("x", "y", "z", "pd", "t1", "t2", "dw")]
    vel = [None] * 3
    if getattr(phantom, "vx", None) is not None:
        vel = [f32(getattr(phantom, k)) for k in ("vx", "vy", "vz")]
    sr = si = None
    if nc:
        sr, si = f32(np.real(sens)), f32(np.imag(sens))
    goff = None if phantom.group_off is None else np.ascontiguousarray(phantom.group_off, np.int64)
    sq = [f64(seq.t), f64(seq.gx), f64(seq.gy), f64(seq.gz), f64(seq.b1.real), f64(seq.b1.imag)]
    adc = np.ascontiguousarray(seq.adc_idx, dtype=np.int64)
    rc = lib.oracle_simulate(float(scanner.gamma), n, *[_p(a) for a in arrs], *[_p(a) for a in vel],
                             nc, _p(sr), _p(si), ng, _p(goff),
                             seq.n_t, *[_p(a) for a in sq], seq.n_adc, _p(adc), int(mode),
                             int(threads or default_threads()), _p(sig), _p(m))
    if rc != 0:
        raise RuntimeError(f"oracle_simulate failed: {rc}")
    s = sig[..., 0] + 1j * sig[..., 1]
    if not nc:
        s = s[0]
    return (s, m) if want_m else s


def excite_step(gamma, m, b1, bz, dt):
    """One excitation-regime rotation of ``m`` = (Mx, My, Mz)."""
    lib = _load()
    mi = np.ascontiguousarray(m, dtype=np.float64)
    mo = np.zeros(3)
    lib.oracle_excite_step(float(gamma), _p(mi), float(np.real(b1)), float(np.imag(b1)),
                           float(bz), float(dt), _p(mo))
    return mo


def relax_step(dt, t1, t2, m0, m):
    lib = _load()
    mi = np.ascontiguousarray(m, dtype=np.float64)
    mo = np.zeros(3)
    lib.oracle_relax_step(float(dt), float(t1), float(t2), float(m0), _p(mi), _p(mo))
    return mo
