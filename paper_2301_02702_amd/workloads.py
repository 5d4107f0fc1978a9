"""Seeded synthetic inputs: scanner, phantoms and discretised sequences.

This module only *builds inputs*. It holds none of the simulation method's
arithmetic (no rotation, precession, relaxation or signal sum), so both the
GPU path and the CPU oracle can be fed from it without sharing any of the
method's code.

Conventions (KomaMRI paper, Methods, "Overview" and "Physical and
Mathematical Background"):

* SI units: positions in m, times in s, gradients in T/m, B1 in T,
  off-resonance ``dw`` in rad/s, gamma in rad/(s T).
* A phantom is a set of independent spins with position (x, y, z), proton
  density ``pd`` (M0), ``t1``, ``t2`` and off-resonance ``dw``. Phantom arrays
  are float32: they are generated in float64 and rounded once, so every
  consumer reads exactly the same values.
* A discretised sequence is a strictly increasing time grid ``t[n_t]``, the
  gradient ``G`` at every grid point (piecewise linear between points), the
  complex RF field ``b1`` per interval (piecewise constant; the paper's
  "concatenation of hard pulses") and the grid indices where the ADC samples.
  An ADC index ``k`` samples the magnetisation at ``t[k]``.
* Spins may be split into signal groups by ``group_off`` (ascending offsets);
  each group gets its own signal, as one dictionary entry of an MRF batch.

Every generator is deterministic in its seed. Proposed values that the
workload description leaves open (timings, FOVs, ellipse layouts) are fixed
here and documented next to the generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Proton gyromagnetic ratio, rad/(s T) (CODATA 2018).
GAMMA = 2.6752218744e8
GAMMA_BAR = GAMMA / (2.0 * np.pi)  # Hz/T


@dataclass
class Scanner:
    b0: float = 1.5
    gamma: float = GAMMA


@dataclass
class Phantom:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    pd: np.ndarray
    t1: np.ndarray
    t2: np.ndarray
    dw: np.ndarray
    group_off: Optional[np.ndarray] = None
    name: str = "phantom"
    # motion: velocities (m/s), position x + v t; None for static spins
    vx: Optional[np.ndarray] = None
    vy: Optional[np.ndarray] = None
    vz: Optional[np.ndarray] = None
    # receive coils: complex sensitivities [n_coils, n] (complex64); None: plain sum
    sens: Optional[np.ndarray] = None

    def __post_init__(self):
        for k in ("x", "y", "z", "pd", "t1", "t2", "dw"):
            setattr(self, k, np.ascontiguousarray(getattr(self, k), dtype=np.float32))
        if self.group_off is not None:
            self.group_off = np.ascontiguousarray(self.group_off, dtype=np.int64)
        if (self.vx is None) != (self.vy is None) or (self.vx is None) != (self.vz is None):
            raise ValueError("give all three velocity components or none")
        if self.vx is not None:
            for k in ("vx", "vy", "vz"):
                setattr(self, k, np.ascontiguousarray(getattr(self, k), dtype=np.float32))
        if self.sens is not None:
            self.sens = np.ascontiguousarray(np.atleast_2d(self.sens), dtype=np.complex64)

    def _extra(self, idx):
        """Motion and coil fields of the spins ``idx``."""
        kw = {}
        if self.vx is not None:
            kw.update(vx=self.vx[idx], vy=self.vy[idx], vz=self.vz[idx])
        if self.sens is not None:
            kw["sens"] = self.sens[:, idx]
        return kw

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_groups(self) -> int:
        return 1 if self.group_off is None else int(self.group_off.shape[0] - 1)

    def subset(self, idx) -> "Phantom":
        """Spins ``idx`` as one group (group structure is dropped)."""
        idx = np.asarray(idx)
        return Phantom(self.x[idx], self.y[idx], self.z[idx], self.pd[idx],
                       self.t1[idx], self.t2[idx], self.dw[idx], None,
                       name=f"{self.name}[subset {idx.shape[0]}]", **self._extra(idx))

    def groups(self, g0: int, g1: int) -> "Phantom":
        """Groups ``g0..g1-1`` with their own offsets."""
        off = self.group_off
        s0, s1 = int(off[g0]), int(off[g1])
        sl = slice(s0, s1)
        return Phantom(self.x[sl], self.y[sl], self.z[sl], self.pd[sl], self.t1[sl],
                       self.t2[sl], self.dw[sl], off[g0:g1 + 1] - s0,
                       name=f"{self.name}[groups {g0}:{g1}]", **self._extra(sl))

    def concat(self, other: "Phantom") -> "Phantom":
        kw = {}
        if self.vx is not None or other.vx is not None:
            v = lambda p, k: getattr(p, k) if p.vx is not None else np.zeros(p.n, np.float32)  # noqa: E731
            kw = {k: np.concatenate([v(self, k), v(other, k)]) for k in ("vx", "vy", "vz")}
        if self.sens is not None or other.sens is not None:
            if self.sens is None or other.sens is None or self.sens.shape[0] != other.sens.shape[0]:
                raise ValueError("both phantoms need sensitivities for the same coils")
            kw["sens"] = np.concatenate([self.sens, other.sens], axis=1)
        return Phantom(*(np.concatenate([getattr(self, k), getattr(other, k)])
                         for k in ("x", "y", "z", "pd", "t1", "t2", "dw")),
                       name=f"{self.name}+{other.name}", **kw)

    @property
    def n_coils(self) -> int:
        return 0 if self.sens is None else int(self.sens.shape[0])

    @property
    def moving(self) -> bool:
        return self.vx is not None


@dataclass
class Sequence:
    t: np.ndarray
    gx: np.ndarray
    gy: np.ndarray
    gz: np.ndarray
    b1: np.ndarray  # complex128, one value per interval
    adc_idx: np.ndarray
    name: str = "sequence"
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        for k in ("t", "gx", "gy", "gz"):
            setattr(self, k, np.ascontiguousarray(getattr(self, k), dtype=np.float64))
        self.b1 = np.ascontiguousarray(self.b1, dtype=np.complex128)
        self.adc_idx = np.ascontiguousarray(self.adc_idx, dtype=np.int64)

    @property
    def n_t(self) -> int:
        return int(self.t.shape[0])

    @property
    def n_int(self) -> int:
        return self.n_t - 1

    @property
    def n_adc(self) -> int:
        return int(self.adc_idx.shape[0])

    @property
    def n_rf(self) -> int:
        return int(np.count_nonzero(self.b1 != 0))

    @property
    def b1_re(self) -> np.ndarray:
        return np.ascontiguousarray(self.b1.real)

    @property
    def b1_im(self) -> np.ndarray:
        return np.ascontiguousarray(self.b1.imag)

    def counts(self, n_spins: int) -> dict:
        return {"n_int": self.n_int, "n_rf": self.n_rf, "n_adc": self.n_adc,
                "spin_steps": int(n_spins) * self.n_int}


# --------------------------------------------------------------------------
# Sequence builder on a uniform raster
# --------------------------------------------------------------------------
class UniformSeq:
    """Builds a sequence on a uniform raster of ``dt`` seconds.

    Gradients live on grid points and are piecewise linear, so a trapezoid
    with ``ramp`` ramp intervals, ``flat`` flat intervals and amplitude ``A``
    has area ``A * (ramp + flat) * dt`` exactly. RF values live on intervals.
    """

    def __init__(self, n_int: int, dt: float):
        self.dt = float(dt)
        self.n_int = int(n_int)
        self.g = np.zeros((3, n_int + 1))
        self.b1 = np.zeros(n_int, dtype=np.complex128)
        self.adc = []

    def trap(self, axis: int, start: int, ramp: int, flat: int, amp: float):
        if ramp < 1 or flat < 0:
            raise ValueError("trapezoid needs ramp >= 1 and flat >= 0")
        i = np.arange(ramp + 1)
        g = self.g[axis]
        g[start:start + ramp + 1] += amp * i / ramp
        g[start + ramp + 1:start + ramp + flat] += amp
        g[start + ramp + flat:start + 2 * ramp + flat + 1] += amp * (ramp - i) / ramp
        if flat == 0:  # the apex point was added by both ramps
            g[start + ramp] -= amp
        return start + 2 * ramp + flat

    def trap_area(self, axis: int, start: int, ramp: int, flat: int, area: float):
        amp = area / ((ramp + flat) * self.dt)
        return self.trap(axis, start, ramp, flat, amp)

    def rf(self, start: int, samples: np.ndarray):
        self.b1[start:start + len(samples)] += samples
        return start + len(samples)

    def adc_points(self, first_point: int, n: int):
        self.adc.extend(range(first_point, first_point + n))

    def build(self, name: str, t0: float = 0.0, **meta) -> Sequence:
        t = t0 + self.dt * np.arange(self.n_int + 1, dtype=np.float64)
        return Sequence(t, self.g[0], self.g[1], self.g[2], self.b1,
                        np.array(self.adc, dtype=np.int64), name=name, meta=meta)


def sinc_pulse(n: int, dt: float, flip: float, lobes: float, gamma: float = GAMMA,
               phase: float = 0.0, freq: float = 0.0) -> np.ndarray:
    """Real sinc envelope sampled at interval midpoints, scaled so that
    ``gamma * sum(B1) * dt = flip`` (net on-resonance flip), times ``exp(i*(phase - 2*pi*freq*(t-tc)))``.

    ``lobes`` is half the time-bandwidth product (the envelope is
    ``sinc(lobes * u)`` for ``u`` in [-1, 1]).
    """
    tm = (np.arange(n) + 0.5) * dt
    tc = n * dt / 2.0
    u = (tm - tc) / tc
    env = np.sinc(lobes * u)
    env = env * flip / (gamma * np.sum(env) * dt)
    return env * np.exp(1j * (phase - 2.0 * np.pi * freq * (tm - tc)))


def hard_pulse(n: int, dt: float, flip: float, gamma: float = GAMMA, phase: float = 0.0):
    amp = flip / (gamma * n * dt)
    return np.full(n, amp * np.exp(1j * phase), dtype=np.complex128)


# --------------------------------------------------------------------------
# Phantoms
# --------------------------------------------------------------------------
def grid_xy(n: int, fov: float):
    """Cell-centred n x n grid over [-fov/2, fov/2)^2; x varies fastest."""
    c = -fov / 2 + (np.arange(n) + 0.5) * (fov / n)
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return xx.ravel(), yy.ravel()


def gre_phantom(seed: int = 1001, n: int = 64, fov: float = 0.2) -> Phantom:
    """64 x 64 grid over 0.2 m, PD = 1, T1 ~ U[0.5, 1.5] s, T2 ~ U[0.05, 0.15] s,
    no off-resonance."""
    rng = np.random.default_rng(seed)
    x, y = grid_xy(n, fov)
    m = x.shape[0]
    return Phantom(x, y, np.zeros(m), np.ones(m), rng.uniform(0.5, 1.5, m),
                   rng.uniform(0.05, 0.15, m), np.zeros(m), name=f"gre_grid{n}")


# tissue classes (PD, T1 s, T2 s)
CLASS_OUTER = (0.8, 1.0, 0.1)
CLASS_INNER = (0.7, 0.6, 0.08)
CLASS_FLUID = (1.0, 4.0, 2.0)
BACKGROUND = (0.0, 1.0, 0.1)


def _ellipse(xx, yy, cx, cy, a, b, theta=0.0):
    c, s = np.cos(theta), np.sin(theta)
    u = (xx - cx) * c + (yy - cy) * s
    v = -(xx - cx) * s + (yy - cy) * c
    return (u / a) ** 2 + (v / b) ** 2 <= 1.0


def head_plane(rng, n: int, fov: float, scale: float, sigma_px: float, dw_std_hz: float):
    """One plane of the head-like phantom: an outer ellipse, an inner ellipse
    and six fluid ellipses, plus a smooth zero-mean Gaussian off-resonance
    field (white noise filtered with a Gaussian of ``sigma_px`` pixels,
    scaled to ``dw_std_hz``, returned in rad/s)."""
    from scipy.ndimage import gaussian_filter

    x, y = grid_xy(n, fov)
    pd = np.full(x.shape, BACKGROUND[0])
    t1 = np.full(x.shape, BACKGROUND[1])
    t2 = np.full(x.shape, BACKGROUND[2])

    def paint(mask, cls):
        pd[mask], t1[mask], t2[mask] = cls

    paint(_ellipse(x, y, 0, 0, 0.090 * scale, 0.110 * scale), CLASS_OUTER)
    paint(_ellipse(x, y, 0, 0, 0.075 * scale, 0.095 * scale), CLASS_INNER)
    for _ in range(6):
        a, b = rng.uniform(0.005, 0.020, 2) * scale
        th = rng.uniform(0, np.pi)
        r = rng.uniform(0, 1) ** 0.5 * 0.5
        ang = rng.uniform(0, 2 * np.pi)
        cx, cy = r * 0.075 * scale * np.cos(ang), r * 0.095 * scale * np.sin(ang)
        paint(_ellipse(x, y, cx, cy, a, b, th), CLASS_FLUID)
    noise = gaussian_filter(rng.standard_normal((n, n)), sigma_px, mode="wrap").ravel()
    noise -= noise.mean()
    noise *= dw_std_hz / noise.std()
    dw = 2.0 * np.pi * noise
    return x, y, pd, t1, t2, dw


def epi_phantom(seed: int = 1002, n: int = 256, fov: float = 0.23) -> Phantom:
    """Head-like 256 x 256 phantom (65,536 spins) over 0.23 m with three tissue
    classes and a smooth off-resonance field of std 50 Hz."""
    rng = np.random.default_rng(seed)
    x, y, pd, t1, t2, dw = head_plane(rng, n, fov, 1.0, 16.0, 50.0)
    return Phantom(x, y, np.zeros_like(x), pd, t1, t2, dw, name=f"epi_head{n}")


SEEPI_NSLICE = 20
SEEPI_SLICE_GAP = 5e-3


def slice_z(s: int) -> float:
    return (s - (SEEPI_NSLICE - 1) / 2.0) * SEEPI_SLICE_GAP


def seepi_phantom(seed: int = 1005, n: int = 500, fov: float = 0.23,
                  n_slices: int = SEEPI_NSLICE) -> Phantom:
    """20 planes of 500 x 500 spins (5e6) at z = (s - 9.5) * 5 mm; the head
    ellipses shrink towards the outer planes; off-resonance std 100 Hz."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in range(n_slices):
        z = slice_z(s)
        scale = np.sqrt(max(0.25, 1.0 - (z / 0.08) ** 2))
        x, y, pd, t1, t2, dw = head_plane(rng, n, fov, scale, 30.0, 100.0)
        parts.append((x, y, np.full_like(x, z), pd, t1, t2, dw))
    cols = [np.concatenate([p[i] for p in parts]) for i in range(7)]
    return Phantom(*cols, name=f"seepi_{n_slices}x{n}")


MRF_NT1 = 100
MRF_NT2 = 100
MRF_ISO = 400
MRF_VOXEL = 1e-3


def mrf_phantom(n_t1: int = MRF_NT1, n_t2: int = MRF_NT2, n_iso: int = MRF_ISO,
                voxel: float = MRF_VOXEL) -> Phantom:
    """Dictionary batch: every (T1, T2) of a log-spaced grid (T1 0.1..4 s,
    T2 0.01..2 s) is one signal group of ``n_iso`` isochromats evenly spaced
    over one voxel along x; PD = 1, no off-resonance."""
    t1v = np.geomspace(0.1, 4.0, n_t1)
    t2v = np.geomspace(0.01, 2.0, n_t2)
    T1, T2 = np.meshgrid(t1v, t2v, indexing="ij")
    n_e = n_t1 * n_t2
    xs = (np.arange(n_iso) + 0.5) * (voxel / n_iso)
    x = np.tile(xs, n_e)
    t1 = np.repeat(T1.ravel(), n_iso)
    t2 = np.repeat(T2.ravel(), n_iso)
    m = x.shape[0]
    off = np.arange(n_e + 1, dtype=np.int64) * n_iso
    ph = Phantom(x, np.zeros(m), np.zeros(m), np.ones(m), t1, t2, np.zeros(m), off,
                 name=f"mrf_{n_t1}x{n_t2}x{n_iso}")
    ph.entries = np.stack([T1.ravel(), T2.ravel()], axis=1)
    return ph


def random_phantom(seed: int, n: int, fov: float = 0.2) -> Phantom:
    """``n`` spins uniform in [-fov/2, fov/2)^2 at z = 0 with the GRE tissue
    distribution (PD = 1, T1 ~ U[0.5, 1.5] s, T2 ~ U[0.05, 0.15] s)."""
    rng = np.random.default_rng(seed)
    f32 = np.float32
    u = lambda lo, hi: rng.random(n, dtype=f32) * f32(hi - lo) + f32(lo)  # noqa: E731  (float32 draws: fast)
    x = u(-fov / 2, fov / 2)
    y = u(-fov / 2, fov / 2)
    return Phantom(x, y, np.zeros(n, f32), np.ones(n, f32), u(0.5, 1.5), u(0.05, 0.15), np.zeros(n, f32),
                   name=f"random{n}")


# --------------------------------------------------------------------------
# Sequences
# --------------------------------------------------------------------------
def gre_sequence(n: int = 64, fov: float = 0.2, dt: float = 10e-6, tr_int: int = 1000,
                 gamma: float = GAMMA) -> Sequence:
    """2D Cartesian gradient echo: per TR (10 ms at dt = 10 us) a 1 ms real
    sinc 90 deg (100 intervals), a 1 ms phase-encode/prephaser, a readout of
    ``n`` ADC samples at 10 us on the flat top of an 11.74 mT/m Gx trapezoid,
    then a Gy rewinder with a Gx spoiler, and idle to the end of the TR."""
    gbar = gamma / (2 * np.pi)
    dk = 1.0 / fov
    s = UniformSeq(n * tr_int, dt)
    g_ro = dk / (gbar * dt)
    ramp = 10
    for line in range(n):
        t0 = line * tr_int
        p = s.rf(t0, sinc_pulse(100, dt, np.pi / 2, 2.0, gamma))
        ky = (line - n // 2) * dk
        kx_pre = -(n // 2) * dk - g_ro * gbar * ramp * dt / 2.0
        s.trap_area(0, p, ramp, 80, kx_pre / gbar)
        s.trap_area(1, p, ramp, 80, ky / gbar)
        p += 100
        flat_start = p + ramp
        s.trap(0, p, ramp, n, g_ro)
        s.adc_points(flat_start, n)
        p = flat_start + n + ramp
        s.trap_area(1, p, ramp, 80, -ky / gbar)
        s.trap(0, p, ramp, 80, 0.020)
    return s.build("gre64", fov=fov, n=n, tr=tr_int * dt)


def _epi_readout(s: UniformSeq, p: int, n: int, fov: float, dt: float, ramp: int,
                 gbar: float, ky_first: int, prephase: int = 100) -> int:
    """Prephaser starting at interval ``p`` then ``n`` EPI lines; returns the
    interval index after the last ramp-down."""
    dk = 1.0 / fov
    g_ro = dk / (gbar * dt)
    ramp_area = g_ro * ramp * dt / 2.0  # area of one ramp, T s/m
    # prephaser: kx to -n/2 dk minus one ramp, ky to ky_first * dk
    kx_pre = -(n // 2) * dk / gbar - ramp_area
    r = 10
    s.trap_area(0, p, r, prephase - 2 * r, kx_pre)
    s.trap_area(1, p, r, prephase - 2 * r, ky_first * dk / gbar)
    p += prephase
    blip_r = 10
    for line in range(n):
        sign = 1.0 if line % 2 == 0 else -1.0
        flat_start = p + ramp
        s.trap(0, p, ramp, n, sign * g_ro)
        s.adc_points(flat_start, n)
        p = flat_start + n + ramp
        if line < n - 1:
            # blip centred on the gap between this flat top and the next
            gap_mid = p  # end of this ramp-down == start of next ramp-up
            s.trap_area(1, gap_mid - blip_r, blip_r, 0, dk / gbar)
    return p


def epi_sequence(n: int = 128, fov: float = 0.23, dt: float = 4e-6, rf_int: int = 50,
                 ramp: int = 15, gamma: float = GAMMA) -> Sequence:
    """Single-shot 2D EPI (dt = 4 us): hard 90 deg of 50 intervals
    (0.2 ms, about 29 uT), a 0.4 ms prephaser, then 128 lines of
    15 ramp + 128 flat (ADC) + 15 ramp intervals with alternating
    +-25.5 mT/m readout and Gy blips of area 1/(gamma_bar FOV)."""
    gbar = gamma / (2 * np.pi)
    n_int = rf_int + 100 + n * (2 * ramp + n)
    s = UniformSeq(n_int, dt)
    p = s.rf(0, hard_pulse(rf_int, dt, np.pi / 2, gamma))
    p = _epi_readout(s, p, n, fov, dt, ramp, gbar, -(n // 2))
    assert p == n_int
    return s.build("epi128", fov=fov, n=n)


def readout_lines_sequence(amps, n_samples: int = 40, ramp: int = 4, dt: float = 4e-6, fov: float = 0.2,
                           gamma: float = GAMMA) -> Sequence:
    """Hard 90 deg, then one flat-top readout line per entry of ``amps``
    (Gx amplitude in T/m; ``n_samples`` ADC points on the flat top), with a
    Gy blip of area 1/(gamma_bar FOV) before every line: lines of equal
    amplitude share their per-sample increments and differ in their start."""
    gbar = gamma / (2 * np.pi)
    per_line = 2 * 2 + 1 + 2 * ramp + n_samples
    n_int = 20 + len(amps) * per_line
    s = UniformSeq(n_int, dt)
    p = s.rf(0, hard_pulse(20, dt, np.pi / 2, gamma))
    for a in amps:
        p = s.trap_area(1, p, 2, 1, 1.0 / (gbar * fov))
        s.adc_points(p + ramp, n_samples)
        p = s.trap(0, p, ramp, n_samples, float(a))
    assert p <= n_int
    return s.build("readout_lines", fov=fov, amps=list(map(float, amps)))


def seepi_sequence(n: int = 128, fov: float = 0.23, dt: float = 4e-6, ramp: int = 15,
                   n_slices: int = SEEPI_NSLICE, te: float = 60e-3,
                   zs=None, gamma: float = GAMMA) -> Sequence:
    """Multi-slice spin-echo EPI (dt = 4 us). Per slice: a slice-selective
    sinc 90 deg (100 intervals, TBW 2, Gz 29.4 mT/m, frequency offset to the
    slice) with a Gz rephaser; a sinc 180 deg along y (200 intervals, TBW 2,
    Gz 14.7 mT/m) centred at TE/2 = 30 ms; an EPI readout as in the single-shot
    EPI with ky ordered so that ky = 0 falls at TE = 60 ms; a 0.4 ms spoiler.
    The next slice follows immediately."""
    gbar = gamma / (2 * np.pi)
    zs = [slice_z(s) for s in range(n_slices)] if zs is None else list(zs)
    line_len = 2 * ramp + n
    r_ss = 10  # slice-select ramps
    g90, g180 = 29.4e-3, 14.7e-3
    # timing (intervals) relative to the 90 deg pulse start
    i90 = r_ss
    c90 = i90 + 50  # centre of the 90
    i180 = c90 + int(round(te / 2 / dt)) - 100 - r_ss  # 180 flat starts so its centre is at TE/2
    c180 = i180 + r_ss + 100
    assert c180 - c90 == int(round(te / 2 / dt))
    ro_start = i180 + 2 * r_ss + 200 + 10  # prephaser start after the 180 ends
    first_flat = ro_start + 100 + ramp
    # as many lines as fit before the ky = 0 line, whose centre sample sits at TE
    te_pt = c90 + int(round(te / dt))
    n_before = (te_pt - first_flat - n // 2) // line_len
    shift = te_pt - (first_flat + n_before * line_len + n // 2)
    assert 0 <= shift < line_len, shift
    ro_start += shift
    slice_len = ro_start + 100 + n * line_len + 100
    s = UniformSeq(slice_len * len(zs), dt)
    for k, z in enumerate(zs):
        b = k * slice_len
        s.trap(2, b, r_ss, 100, g90)
        s.rf(b + i90, sinc_pulse(100, dt, np.pi / 2, 1.0, gamma, 0.0, gbar * g90 * z))
        # rephase the second half of the slice select (flat half + ramp)
        reph_area = -(g90 * (50 + r_ss / 2.0) * dt)
        s.trap_area(2, b + i90 + 100 + r_ss, 10, 60, reph_area)
        s.trap(2, b + i180, r_ss, 200, g180)
        s.rf(b + i180 + r_ss, sinc_pulse(200, dt, np.pi, 1.0, gamma, np.pi / 2,
                                         gbar * g180 * z))
        p = _epi_readout(s, b + ro_start, n, fov, dt, ramp, gbar, -n_before)
        s.trap(0, p, 10, 80, 0.02)
        s.trap(2, p, 10, 80, 0.02)
    return s.build(f"seepi{len(zs)}", fov=fov, n=n, te=te, zs=zs)


def mrf_sequence(seed: int = 2004, n_tr: int = 1000, voxel: float = MRF_VOXEL,
                 gamma: float = GAMMA) -> Sequence:
    """FISP fingerprinting train on a sequence-aware (non-uniform) grid:
    1000 TRs, TR ~ U[12, 15] ms on a 10 us raster; flip
    37.5 + 32.5 sin(2 pi n / P + psi) deg (5..70 deg), P ~ U[200, 400],
    psi ~ U[0, 2 pi); hard RF of 10 x 10 us; one ADC 5 ms after the RF centre;
    a Gx spoiler (0.1/0.8/0.1 ms) of area 1/(gamma_bar voxel) starting 6 ms
    after the RF start. 16 intervals per TR."""
    rng = np.random.default_rng(seed)
    gbar = gamma / (2 * np.pi)
    raster = 10e-6
    tr = np.round(rng.uniform(12e-3, 15e-3, n_tr) / raster) * raster
    period = rng.uniform(200, 400)
    psi = rng.uniform(0, 2 * np.pi)
    nn = np.arange(n_tr)
    flip = np.deg2rad(37.5 + 32.5 * np.sin(2 * np.pi * nn / period + psi))
    g_sp = 1.0 / (gbar * voxel) / 0.9e-3
    t, gx, b1, adc = [], [], [], []
    t0 = 0.0
    for k in range(n_tr):
        rel = [i * 10e-6 for i in range(11)] + [5.05e-3, 6.0e-3, 6.1e-3, 6.9e-3, 7.0e-3]
        g = [0.0] * 11 + [0.0, 0.0, g_sp, g_sp, 0.0]
        amp = flip[k] / (gamma * 100e-6)
        rf = [amp] * 10 + [0.0] * 6
        for i, (r, gg) in enumerate(zip(rel, g)):
            if i == 11:
                adc.append(len(t))
            t.append(t0 + r)
            gx.append(gg)
        b1.extend(rf)
        t0 += tr[k]
    t.append(t0)
    gx.append(0.0)
    t = np.array(t)
    z = np.zeros_like(t)
    return Sequence(t, np.array(gx), z, z, np.array(b1, dtype=np.complex128),
                    np.array(adc), name="mrf_fisp1000",
                    meta={"flip": flip, "tr": tr, "period": period, "psi": psi})


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------
def config(k: int):
    """Return (scanner, phantom, sequence) of workload ``k`` in 1..5
    (serving, k = 3, is generated per request by :func:`serving_requests`)."""
    sc = Scanner()
    if k == 1:
        return sc, gre_phantom(), gre_sequence()
    if k == 2:
        return sc, epi_phantom(), epi_sequence()
    if k == 4:
        return sc, mrf_phantom(), mrf_sequence()
    if k == 5:
        return sc, seepi_phantom(), seepi_sequence()
    raise ValueError("serving workload: use serving_requests()")


WORKLOAD_NAMES = {
    1: "gre64 (64x64 grid, 64 TR x 1000 int, 4096 ADC)",
    2: "epi256 (256x256 head, 128x128 EPI, 20374 int)",
    3: "serving_mix (1e3-1e6 spins, GRE/EPI/SE-EPI slice)",
    4: "mrf_fisp (100x100 T1/T2 x 400 iso, 1000 TR)",
    5: "seepi20x500 (5e6 spins, 20 slices, 327680 ADC)",
}


@dataclass
class ServingRequest:
    rid: int
    arrival: float  # seconds after the stream start (unit mean gap, scaled by caller)
    n_spins: int
    kind: str  # "gre" | "epi" | "seepi"
    phantom_seed: int


def serving_requests(n: int = 1000, seed: int = 3000, lo: float = 3.0, hi: float = 6.0):
    """Requests with log-uniform phantom sizes 10^U(lo, hi) spins, a
    sequence kind drawn uniformly from {GRE, EPI, one SE-EPI slice at z = 0}
    and unit-mean exponential inter-arrival gaps (multiply by 1/lambda)."""
    rng = np.random.default_rng(seed)
    sizes = np.round(10.0 ** rng.uniform(lo, hi, n)).astype(np.int64)
    kinds = rng.choice(["gre", "epi", "seepi"], n)
    gaps = rng.exponential(1.0, n)
    arr = np.cumsum(gaps) - gaps[0]
    return [ServingRequest(i, float(arr[i]), int(sizes[i]), str(kinds[i]), seed * 10 + i)
            for i in range(n)]


_SEQ_CACHE = {}


def serving_sequence(kind: str) -> Sequence:
    if kind not in _SEQ_CACHE:
        if kind == "gre":
            _SEQ_CACHE[kind] = gre_sequence()
        elif kind == "epi":
            _SEQ_CACHE[kind] = epi_sequence()
        elif kind == "seepi":
            _SEQ_CACHE[kind] = seepi_sequence(zs=[0.0])
        else:
            raise ValueError(kind)
    return _SEQ_CACHE[kind]


def serving_phantom(req: ServingRequest) -> Phantom:
    return random_phantom(req.phantom_seed, req.n_spins)


# --------------------------------------------------------------------------
# Small sequences used by the closed-form and property tests
# --------------------------------------------------------------------------
def make_sequence(t, g, b1, adc_idx, name="custom") -> Sequence:
    """Sequence from explicit arrays; ``g`` is (n_t, 3)."""
    g = np.asarray(g, dtype=np.float64).reshape(-1, 3)
    return Sequence(np.asarray(t, dtype=np.float64), g[:, 0], g[:, 1], g[:, 2],
                    np.asarray(b1, dtype=np.complex128), np.asarray(adc_idx), name=name)


def single_spin(x=0.0, y=0.0, z=0.0, pd=1.0, t1=np.inf, t2=np.inf, dw=0.0) -> Phantom:
    a = lambda v: np.array([v], dtype=np.float64)  # noqa: E731
    return Phantom(a(x), a(y), a(z), a(pd), a(t1), a(t2), a(dw), name="spin")


def random_sequence(rng, n_int: int, p_rf: float = 0.5, b1_max: float = 2e-5,
                    g_max: float = 0.03, dt_range=(1e-6, 1e-4), p_adc: float = 0.3) -> Sequence:
    """Random grid with random piecewise-linear G, random complex B1 on a
    fraction ``p_rf`` of the intervals and random ADC points."""
    dt = rng.uniform(*dt_range, n_int)
    t = np.concatenate([[0.0], np.cumsum(dt)])
    g = rng.uniform(-g_max, g_max, (n_int + 1, 3))
    rf = rng.uniform(size=n_int) < p_rf
    b1 = np.where(rf, rng.uniform(-b1_max, b1_max, n_int) + 1j * rng.uniform(-b1_max, b1_max, n_int), 0)
    adc = np.nonzero(rng.uniform(size=n_int + 1) < p_adc)[0]
    return make_sequence(t, g, b1, adc, name=f"random{n_int}")


def random_spins(rng, n: int, extent: float = 0.1, dw_max: float = 2000.0,
                 finite_t: bool = True) -> Phantom:
    x, y, z = rng.uniform(-extent, extent, (3, n))
    pd = rng.uniform(0.2, 1.0, n)
    if finite_t:
        t1 = rng.uniform(0.05, 3.0, n)
        t2 = rng.uniform(0.01, 1.0, n) * np.minimum(1.0, t1)
    else:
        t1 = np.full(n, np.inf)
        t2 = np.full(n, np.inf)
    dw = rng.uniform(-dw_max, dw_max, n)
    return Phantom(x, y, z, pd, t1, t2, dw, name=f"random_spins{n}")


def fourier_sequence(n: int = 64, fov: float = 0.2, dt: float = 10e-6, rf_dt: float = 1e-6,
                     gamma: float = GAMMA) -> Sequence:
    """One single-interval hard 90 deg (``rf_dt`` long) followed by a
    Cartesian multi-line readout without re-excitation: for every line a
    prephaser to (kx, ky) = (-n/2, line - n/2) / FOV, ``n`` ADC samples on a
    flat Gx giving Delta k = 1/FOV per sample, then a rewinder to k = 0."""
    gbar = gamma / (2 * np.pi)
    dk = 1.0 / fov
    g_ro = dk / (gbar * dt)
    ramp = 10
    line_int = 100 + 2 * ramp + n + 100
    s = UniformSeq(line_int * n, dt)
    for line in range(n):
        p = line * line_int
        ky = (line - n // 2) * dk
        kx_pre = -(n // 2) * dk - g_ro * gbar * ramp * dt / 2.0
        s.trap_area(0, p, ramp, 80, kx_pre / gbar)
        s.trap_area(1, p, ramp, 80, ky / gbar)
        p += 100
        s.trap(0, p, ramp, n, g_ro)
        s.adc_points(p + ramp, n)
        p += 2 * ramp + n
        kx_end = kx_pre + g_ro * gbar * (ramp + n) * dt
        s.trap_area(0, p, ramp, 80, -kx_end / gbar)
        s.trap_area(1, p, ramp, 80, -ky / gbar)
    seq = s.build("fourier", t0=rf_dt, fov=fov, n=n)
    # prepend the single RF interval [0, rf_dt]
    t = np.concatenate([[0.0], seq.t])
    gx = np.concatenate([[0.0], seq.gx])
    gy = np.concatenate([[0.0], seq.gy])
    gz = np.concatenate([[0.0], seq.gz])
    b1 = np.concatenate([hard_pulse(1, rf_dt, np.pi / 2, gamma), seq.b1])
    return Sequence(t, gx, gy, gz, b1, seq.adc_idx + 1, name="fourier", meta=seq.meta)


def epi_te_sequence(n: int = 100, fov: float = 0.23, te: float = 0.1, dt: float = 4e-6,
                    rf_int: int = 1, ramp: int = 15, gamma: float = GAMMA) -> Sequence:
    """Single-shot gradient-echo EPI whose k = (0, 0) sample (line n/2,
    sample n/2) lies exactly ``te`` after the centre of a hard 90 deg pulse of
    ``rf_int`` intervals; ``n`` x ``n`` samples with Delta k = 1/FOV."""
    gbar = gamma / (2 * np.pi)
    line_len = 2 * ramp + n
    k0_rel = 100 + ramp + (n // 2) * line_len + n // 2
    te_int = int(round(te / dt))
    # te is measured from the pulse centre; with an odd rf_int the centre is
    # rounded down to a grid point (rf_int = 1: te is measured from the start)
    p_ro = te_int + rf_int // 2 - k0_rel
    if p_ro < rf_int:
        raise ValueError("te too short for this readout")
    n_int = p_ro + 100 + n * line_len
    s = UniformSeq(n_int, dt)
    s.rf(0, hard_pulse(rf_int, dt, np.pi / 2, gamma))
    end = _epi_readout(s, p_ro, n, fov, dt, ramp, gbar, -(n // 2))
    assert end == n_int
    k0_point = p_ro + k0_rel
    return s.build(f"epi{n}_te{te * 1e3:g}ms", fov=fov, n=n, te=te,
                   k0_adc=int(np.searchsorted(np.array(s.adc), k0_point)), k0_point=k0_point)


# --------------------------------------------------------------------------
# Block-structured sequences (input of the sequence-aware discretiser)
# --------------------------------------------------------------------------
# A sequence is a list of blocks played back to back; times inside a block
# are relative to its start. Gradients are trapezoids or piecewise-linear
# waveforms through given vertices, RF is a train of piecewise-constant
# samples, the ADC samples at delay + i * dwell.
@dataclass
class Trap:
    amp: float  # T/m
    delay: float
    rise: float
    flat: float
    fall: float


@dataclass
class PWL:
    t: np.ndarray    # block-local vertex times, s
    amp: np.ndarray  # T/m


@dataclass
class RFTrain:
    delay: float
    dt: float
    samples: np.ndarray  # complex, T


@dataclass
class ADCWindow:
    delay: float
    dwell: float
    n: int


@dataclass
class Block:
    duration: float
    gx: Optional[object] = None
    gy: Optional[object] = None
    gz: Optional[object] = None
    rf: Optional[RFTrain] = None
    adc: Optional[ADCWindow] = None

    @property
    def grads(self):
        return (self.gx, self.gy, self.gz)


def trap_of_area(area: float, ramp: float, flat: float, delay: float = 0.0) -> Trap:
    """Trapezoid of ``area`` T s/m (area = amp * (ramp + flat))."""
    return Trap(area / (ramp + flat), delay, ramp, flat, ramp)


def gre_blocks(n: int = 64, fov: float = 0.2, dt: float = 10e-6, tr_int: int = 1000,
               gamma: float = GAMMA):
    """The gradient echo of :func:`gre_sequence` as blocks: per TR an RF
    block, a prephaser / phase-encode block, a readout block, a rewinder /
    spoiler block and an idle block, with the same timings on the same raster."""
    gbar = gamma / (2 * np.pi)
    dk = 1.0 / fov
    g_ro = dk / (gbar * dt)
    ramp = 10
    blocks = []
    for line in range(n):
        ky = (line - n // 2) * dk
        kx_pre = -(n // 2) * dk - g_ro * gbar * ramp * dt / 2.0
        blocks.append(Block(100 * dt, rf=RFTrain(0.0, dt, sinc_pulse(100, dt, np.pi / 2, 2.0, gamma))))
        blocks.append(Block(100 * dt, gx=trap_of_area(kx_pre / gbar, ramp * dt, 80 * dt),
                            gy=trap_of_area(ky / gbar, ramp * dt, 80 * dt)))
        blocks.append(Block((2 * ramp + n) * dt, gx=Trap(g_ro, 0.0, ramp * dt, n * dt, ramp * dt),
                            adc=ADCWindow(ramp * dt, dt, n)))
        blocks.append(Block(100 * dt, gx=Trap(0.020, 0.0, ramp * dt, 80 * dt, ramp * dt),
                            gy=trap_of_area(-ky / gbar, ramp * dt, 80 * dt)))
        blocks.append(Block((tr_int - 300 - (2 * ramp + n)) * dt))
    return blocks


def epi_blocks(n: int = 128, fov: float = 0.23, dt: float = 4e-6, rf_int: int = 50,
               ramp: int = 15, gamma: float = GAMMA):
    """The single-shot EPI of :func:`epi_sequence` as blocks: an RF block, a
    prephaser block and one block per line. Each Gy blip straddles two line
    blocks, so the line blocks carry its halves as piecewise-linear
    waveforms that meet at the boundary with the blip's peak."""
    gbar = gamma / (2 * np.pi)
    dk = 1.0 / fov
    g_ro = dk / (gbar * dt)
    ramp_area = g_ro * ramp * dt / 2.0
    kx_pre = -(n // 2) * dk / gbar - ramp_area
    blip_r = 10
    blip_amp = (dk / gbar) / (blip_r * dt)
    dur = (2 * ramp + n) * dt
    blocks = [Block(rf_int * dt, rf=RFTrain(0.0, dt, hard_pulse(rf_int, dt, np.pi / 2, gamma))),
              Block(100 * dt, gx=trap_of_area(kx_pre, 10 * dt, 80 * dt),
                    gy=trap_of_area(-(n // 2) * dk / gbar, 10 * dt, 80 * dt))]
    for line in range(n):
        sign = 1.0 if line % 2 == 0 else -1.0
        tv, av = [], []
        if line > 0:  # falling half of the previous blip
            tv += [0.0, blip_r * dt]
            av += [blip_amp, 0.0]
        if line < n - 1:  # rising half of the next blip
            tv += [dur - blip_r * dt, dur]
            av += [0.0, blip_amp]
        gy = PWL(np.array(tv), np.array(av)) if tv else None
        blocks.append(Block(dur, gx=Trap(sign * g_ro, 0.0, ramp * dt, n * dt, ramp * dt), gy=gy,
                            adc=ADCWindow(ramp * dt, dt, n)))
    return blocks


def random_blocks(rng, n_blocks: int, p_rf: float = 0.4, p_adc: float = 0.5, g_max: float = 0.03,
                  b1_max: float = 2e-5):
    """Random block sequence off any raster: trapezoids, piecewise-linear
    waveforms (some meeting the next block with a non-zero value), RF trains
    and ADC windows at random offsets."""
    blocks = []
    carry = [0.0, 0.0, 0.0]  # G each axis must start from (continuity)
    for b in range(n_blocks):
        dur = rng.uniform(0.2e-3, 2e-3)
        grads = []
        nxt = [0.0, 0.0, 0.0]
        for a in range(3):
            kind = rng.integers(0, 3) if carry[a] == 0.0 else 2
            if kind == 0:
                grads.append(None)
            elif kind == 1:
                rise, fall = rng.uniform(0.02, 0.2, 2) * dur
                flat = rng.uniform(0.0, 0.3) * dur
                delay = rng.uniform(0.0, dur - rise - flat - fall)
                grads.append(Trap(rng.uniform(-g_max, g_max), delay, rise, flat, fall))
            else:
                m = int(rng.integers(2, 7))
                ends_at_end = b + 1 < n_blocks and rng.uniform() < 0.5
                starts_at_0 = carry[a] != 0.0
                t0 = 0.0 if starts_at_0 else rng.uniform(0.0, 0.3) * dur
                t1 = dur if ends_at_end else rng.uniform(0.7, 1.0) * dur
                tv = np.sort(np.concatenate([[t0, t1], rng.uniform(t0, t1, m - 2)]))
                av = rng.uniform(-g_max, g_max, m)
                av[0] = carry[a] if starts_at_0 else 0.0
                av[-1] = av[-1] if ends_at_end else 0.0
                if ends_at_end:
                    nxt[a] = av[-1]
                grads.append(PWL(tv, av))
        carry = nxt
        rf = None
        if rng.uniform() < p_rf:
            k = int(rng.integers(1, 20))
            dt = rng.uniform(2e-6, 40e-6)
            delay = rng.uniform(0.0, max(dur - k * dt, 0.0))
            if delay + k * dt <= dur:
                rf = RFTrain(delay, dt, rng.uniform(-b1_max, b1_max, k) + 1j * rng.uniform(-b1_max, b1_max, k))
        adc = None
        if rng.uniform() < p_adc:
            k = int(rng.integers(1, 40))
            dwell = rng.uniform(3e-6, 30e-6)
            delay = rng.uniform(0.0, max(dur - (k - 1) * dwell, 0.0))
            if delay + (k - 1) * dwell <= dur:
                adc = ADCWindow(delay, dwell, k)
        blocks.append(Block(dur, *grads, rf=rf, adc=adc))
    return blocks


# --------------------------------------------------------------------------
# Motion and receive coils
# --------------------------------------------------------------------------
def with_velocity(ph: Phantom, v=(0.0, 0.1, 0.0), spread: float = 0.0, seed: int = 0) -> Phantom:
    """The phantom moving with velocity ``v`` (m/s), position x + v t; the
    paper's motion example is u_y = v_y t with v_y = 0.1 m/s. ``spread``
    adds a seeded per-spin Gaussian velocity of that standard deviation."""
    rng = np.random.default_rng(seed)
    vel = [np.full(ph.n, float(c)) + (spread * rng.normal(size=ph.n) if spread else 0.0) for c in v]
    out = Phantom(ph.x, ph.y, ph.z, ph.pd, ph.t1, ph.t2, ph.dw, ph.group_off, name=f"{ph.name}+motion",
                  vx=vel[0], vy=vel[1], vz=vel[2], sens=ph.sens)
    return out


def coil_sensitivities(ph: Phantom, n_coils: int = 8, radius: float = 0.16, width: float = 0.12) -> np.ndarray:
    """Synthetic smooth receive sensitivities [n_coils, n] (complex64): coils
    evenly spaced on a circle of ``radius`` in the xy plane around the FOV,
    magnitude falling off with distance as 1 / (1 + (d / width)^2), phase
    turning with the angle seen from the coil (a loop-coil-like field)."""
    ang = 2 * np.pi * np.arange(n_coils) / n_coils
    cx, cy = radius * np.cos(ang), radius * np.sin(ang)
    dx = ph.x.astype(np.float64)[None, :] - cx[:, None]
    dy = ph.y.astype(np.float64)[None, :] - cy[:, None]
    dz = ph.z.astype(np.float64)[None, :]
    d2 = dx * dx + dy * dy + dz * dz
    mag = 1.0 / (1.0 + d2 / width ** 2)
    phase = np.arctan2(dy, dx) - ang[:, None]
    return (mag * np.exp(1j * phase)).astype(np.complex64)


def with_coils(ph: Phantom, n_coils: int = 8, **kw) -> Phantom:
    out = Phantom(ph.x, ph.y, ph.z, ph.pd, ph.t1, ph.t2, ph.dw, ph.group_off, name=f"{ph.name}+{n_coils}coils",
                  vx=ph.vx, vy=ph.vy, vz=ph.vz, sens=coil_sensitivities(ph, n_coils, **kw))
    return out
