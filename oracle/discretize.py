"""Plain reference of sequence-aware time stepping.

TEST INFRASTRUCTURE ONLY: the tests use it to check the library's
discretiser; the product never imports it, and it shares no code with the
library.

Section "Simulation blocks, Regime Switching, and Sequence-Aware Time
Stepping": the phase of a precession interval is integrated with the
trapezoidal rule, which is exact for a gradient that is linear on the
interval, so a grid holding every vertex of G loses nothing; B1 is taken
piecewise constant (a train of hard pulses), for which the spinor rotation
of Eq. Rot_exc is exact on each sample, so a grid holding every RF sample
boundary loses nothing either. Extra points are needed only where the ADC
samples. The paper's two user knobs bound the step between intermediate
gradient points (Delta t, ``dt_max``) and between RF points (Delta t_rf,
``dt_rf_max``).

Readings (the paper does not spell these out):
  * blocks are played back to back from t = 0; event times are block-local;
  * block boundaries are always grid points;
  * an RF sample longer than ``dt_rf_max`` is cut into equal parts; an
    interval outside RF longer than ``dt_max`` is cut into equal parts;
  * points closer than 1 ps are one point (ADC flags are kept);
  * B1 of an interval is the RF sample in force at its midpoint, else 0.

The input is a list of block descriptions (``workloads.Block``).
"""
from __future__ import annotations

import math

import numpy as np

MERGE_TOL = 1e-12  # s


def _vertices(g):
    """(times, amplitudes) of one gradient axis, block-local, or None."""
    if g is None:
        return None
    if hasattr(g, "rise"):  # trapezoid
        t = [g.delay, g.delay + g.rise, g.delay + g.rise + g.flat, g.delay + g.rise + g.flat + g.fall]
        return np.array(t), np.array([0.0, g.amp, g.amp, 0.0])
    return np.asarray(g.t, dtype=np.float64), np.asarray(g.amp, dtype=np.float64)


def _grad(g, u):
    """Gradient of one axis at block-local time u (linear between vertices, 0 outside)."""
    v = _vertices(g)
    if v is None:
        return 0.0
    t, a = v
    if u < t[0] - MERGE_TOL or u > t[-1] + MERGE_TOL:
        return 0.0
    return float(np.interp(u, t, a))


def discretize(blocks, dt_max: float = math.inf, dt_rf_max: float = math.inf):
    """Return (t, g[n_t, 3], b1[n_t - 1] complex, adc_idx)."""
    starts = [0.0]
    for b in blocks:
        starts.append(starts[-1] + b.duration)

    # every time the method needs, with an ADC flag
    pts = []
    for k, b in enumerate(blocks):
        T = starts[k]
        pts.append((T, False))
        for g in b.grads:
            v = _vertices(g)
            if v is not None:
                pts += [(T + float(tv), False) for tv in v[0]]
        if b.rf is not None and len(b.rf.samples) > 0:
            n = len(b.rf.samples)
            parts = 1 if math.isinf(dt_rf_max) else max(1, math.ceil((b.rf.dt - MERGE_TOL) / dt_rf_max))
            for i in range(n):
                for j in range(parts):
                    pts.append((T + b.rf.delay + b.rf.dt * (i + j / parts), False))
            pts.append((T + b.rf.delay + b.rf.dt * n, False))
        if b.adc is not None:
            pts += [(T + b.adc.delay + b.adc.dwell * i, True) for i in range(b.adc.n)]
    pts.append((starts[-1], False))
    pts.sort(key=lambda p: p[0])

    merged = []
    for tp, adc in pts:
        if merged and tp - merged[-1][0] <= MERGE_TOL:
            if adc and merged[-1][1]:
                raise ValueError("two ADC samples at one instant")
            merged[-1][1] = merged[-1][1] or adc
        else:
            merged.append([tp, adc])

    def block_at(tm):
        k = int(np.searchsorted(starts, tm, side="right")) - 1
        return min(max(k, 0), len(blocks) - 1)

    def rf_at(tm):
        k = block_at(tm)
        rf = blocks[k].rf
        if rf is None or len(rf.samples) == 0:
            return None
        i = math.floor((tm - starts[k] - rf.delay) / rf.dt)
        return complex(rf.samples[i]) if 0 <= i < len(rf.samples) else None

    grid = []
    for i, (tp, adc) in enumerate(merged):
        grid.append((tp, adc))
        if i + 1 < len(merged) and not math.isinf(dt_max):
            nxt = merged[i + 1][0]
            if nxt - tp > dt_max and rf_at(0.5 * (tp + nxt)) is None:
                parts = math.ceil((nxt - tp - MERGE_TOL) / dt_max)
                grid += [(tp + (nxt - tp) * (j / parts), False) for j in range(1, parts)]

    t = np.array([p[0] for p in grid])
    g = np.zeros((len(t), 3))
    for i, tm in enumerate(t):
        k = block_at(tm)
        for a, ga in enumerate(blocks[k].grads):
            g[i, a] = _grad(ga, tm - starts[k])
    b1 = np.zeros(len(t) - 1, dtype=np.complex128)
    for i in range(len(t) - 1):
        v = rf_at(0.5 * (t[i] + t[i + 1]))
        b1[i] = 0.0 if v is None else v
    adc_idx = np.array([i for i, p in enumerate(grid) if p[1]], dtype=np.int64)
    return t, g, b1, adc_idx
