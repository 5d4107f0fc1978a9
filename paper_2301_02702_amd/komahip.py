"""Thin ctypes binding of ``libkomahip.so`` (see ``include/komahip.h``).

Argument marshalling only: every step of the simulation runs in the HIP
library. The ``koma_*`` functions mirror the C entry points one to one;
``Context`` and ``Request`` wrap them for numpy / torch callers. Importing
this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkomahip.so")

KOMA_OK = 0
KOMA_E_BUDGET = -5
STATUS = {0: "KOMA_OK", -1: "KOMA_E_ARG", -2: "KOMA_E_PHANTOM", -3: "KOMA_E_SEQUENCE",
          -4: "KOMA_E_NOMEM", -5: "KOMA_E_BUDGET", -6: "KOMA_E_DEVICE", -7: "KOMA_E_CANCELLED",
          -8: "KOMA_E_STATE"}
KOMA_FP64, KOMA_MIXED = 0, 1
KOMA_HOST, KOMA_DEVICE = 0, 1
KERNEL_KINDS = {"seq": 0, "par": 1, "reduce": 2, "aux": 3, "mrf": 4}


class KomaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class koma_scanner(ctypes.Structure):
    _fields_ = [("b0", c_double), ("gamma", c_double)]


class koma_phantom(ctypes.Structure):
    _fields_ = [("n", c_int64), ("x", c_void_p), ("y", c_void_p), ("z", c_void_p), ("pd", c_void_p),
                ("t1", c_void_p), ("t2", c_void_p), ("dw", c_void_p), ("n_groups", c_int64),
                ("group_off", c_void_p), ("vx", c_void_p), ("vy", c_void_p), ("vz", c_void_p),
                ("n_coils", c_int64), ("sens_re", c_void_p), ("sens_im", c_void_p)]


class koma_sequence(ctypes.Structure):
    _fields_ = [("n_t", c_int64), ("t", c_void_p), ("gx", c_void_p), ("gy", c_void_p),
                ("gz", c_void_p), ("b1_re", c_void_p), ("b1_im", c_void_p), ("n_adc", c_int64),
                ("adc_idx", c_void_p)]


class koma_config(ctypes.Structure):
    _fields_ = [("precision", c_int), ("spins_per_lane", c_int), ("wg_size", c_int),
                ("chunk_events", c_int64), ("hbm_budget", c_size_t), ("partial_budget", c_size_t),
                ("defer_min_adc", c_int), ("stretch_max", c_int), ("sample_engine", c_int),
                ("tile_packing", c_int), ("lanes_per_spin", c_int), ("stretches_per_wg", c_int)]


class koma_req_info(ctypes.Structure):
    _fields_ = [(k, c_int64) for k in (
        "n_spins", "n_tiles", "n_groups", "n_adc", "n_events", "n_rf", "n_rf_events", "n_runs", "n_inline_adc",
        "n_deferred_adc", "n_stretches", "n_families", "n_snapshots", "n_blocks", "spins_per_lane", "n_chunks",
        "events_done")] + [("footprint", c_size_t), ("n_ends", c_int64), ("n_rf_in_runs", c_int64),
                           ("n_rows", c_int64), ("lanes_per_spin", c_int64), ("max_single_run", c_int64),
                           ("stretches_per_wg", c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class koma_trap(ctypes.Structure):
    _fields_ = [("amp", c_double), ("delay", c_double), ("rise", c_double), ("flat", c_double),
                ("fall", c_double)]


class koma_grad(ctypes.Structure):
    _fields_ = [("kind", c_int), ("trap", koma_trap), ("pwl_n", c_int64), ("pwl_t", c_void_p),
                ("pwl_amp", c_void_p)]


class koma_rf(ctypes.Structure):
    _fields_ = [("delay", c_double), ("dt", c_double), ("n", c_int64), ("re", c_void_p), ("im", c_void_p)]


class koma_adc(ctypes.Structure):
    _fields_ = [("delay", c_double), ("dwell", c_double), ("n", c_int64)]


class koma_block(ctypes.Structure):
    _fields_ = [("duration", c_double), ("g", koma_grad * 3), ("rf", koma_rf), ("adc", koma_adc)]


KOMA_GRAD_NONE, KOMA_GRAD_TRAP, KOMA_GRAD_PWL = 0, 1, 2

EXPORTS = {
    "koma_config_default": (None, [POINTER(koma_config)]),
    "koma_ctx_create": (c_int, [c_int, POINTER(koma_config), POINTER(c_void_p)]),
    "koma_ctx_destroy": (None, [c_void_p]),
    "koma_last_error": (c_char_p, [c_void_p]),
    "koma_ctx_set_config": (c_int, [c_void_p, POINTER(koma_config)]),
    "koma_footprint": (c_int, [POINTER(koma_phantom), POINTER(koma_sequence), POINTER(koma_config),
                               POINTER(c_size_t)]),
    "koma_simulate": (c_int, [c_void_p, POINTER(koma_scanner), POINTER(koma_phantom),
                              POINTER(koma_sequence), c_int, c_void_p, c_void_p, c_void_p]),
    "koma_simulate_async": (c_int, [c_void_p, POINTER(koma_scanner), POINTER(koma_phantom),
                                    POINTER(koma_sequence), c_void_p, c_void_p, c_void_p, c_void_p]),
    "koma_simulate_noalloc": (c_int, [c_void_p, POINTER(koma_scanner), POINTER(koma_phantom),
                                      POINTER(koma_sequence), c_void_p, c_void_p, c_void_p, c_void_p]),
    "koma_noalloc_capacity": (c_size_t, []),
    "koma_req_open": (c_int, [c_void_p, POINTER(koma_scanner), POINTER(koma_phantom),
                              POINTER(koma_sequence), c_int, POINTER(c_void_p)]),
    "koma_req_advance": (c_int, [c_void_p, c_int64, c_void_p]),
    "koma_req_done": (c_int, [c_void_p, POINTER(c_int)]),
    "koma_req_result": (c_int, [c_void_p, c_void_p, c_void_p]),
    "koma_req_save": (c_int, [c_void_p, c_void_p, POINTER(c_size_t)]),
    "koma_req_load": (c_int, [c_void_p, c_void_p, c_size_t]),
    "koma_req_close": (None, [c_void_p]),
    "koma_req_info_get": (c_int, [c_void_p, POINTER(koma_req_info)]),
    "koma_plan_info": (c_int, [POINTER(koma_scanner), POINTER(koma_phantom), POINTER(koma_sequence),
                               POINTER(koma_config), POINTER(koma_req_info)]),
    "koma_ctx_profile": (c_int, [c_void_p, c_int]),
    "koma_ctx_mem": (c_int, [c_void_p, POINTER(c_size_t), POINTER(c_size_t), POINTER(c_size_t)]),
    "koma_ctx_kernel_stats": (c_int, [c_void_p, c_int, POINTER(c_double), POINTER(c_int64),
                                      POINTER(c_int64)]),
    "koma_discretize": (c_int, [POINTER(koma_block), c_int64, c_double, c_double, POINTER(c_int64),
                                POINTER(c_int64)] + [c_void_p] * 7),
    "koma_mrf_match": (c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_int64, c_int, c_void_p,
                               c_void_p, c_void_p]),
    "koma_mrf_svd": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_int, c_int, c_int, c_int, c_void_p,
                             c_void_p, c_void_p]),
    "koma_mrf_project": (c_int, [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_int, c_int, c_void_p,
                                 c_void_p]),
}

_lib = None


def lib():
    """Load the library; raise if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        try:
            # torch ships its own HIP runtime under the same soname; loading it
            # first makes this library bind to it, so the process holds one
            # runtime and torch's device memory and streams are valid here
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2301_02702_amd.build` (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != KOMA_OK:
        msg = lib().koma_last_error(ctx)
        raise KomaError(status, msg.decode() if msg else "")


# ---------------------------------------------------------------- marshalling
def _ptr(a):
    """Pointer of a numpy array or torch tensor (None stays NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


def make_config(precision="mixed", **kw) -> koma_config:
    c = koma_config()
    lib().koma_config_default(ctypes.byref(c))
    c.precision = {"fp64": KOMA_FP64, "mixed": KOMA_MIXED}[precision] if isinstance(precision, str) else precision
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def make_scanner(scanner) -> koma_scanner:
    return koma_scanner(float(scanner.b0), float(scanner.gamma))


class _PhantomArgs:
    """Holds the arrays (numpy host arrays or torch device tensors) alive."""

    KEYS = ("x", "y", "z", "pd", "t1", "t2", "dw")
    VEL = ("vx", "vy", "vz")

    def __init__(self, phantom, device: bool):
        self.keep = []
        get = (lambda k: phantom.get(k)) if isinstance(phantom, dict) else (lambda k: getattr(phantom, k, None))
        moving = get("vx") is not None
        keys = self.KEYS + (self.VEL if moving else ())
        if device:
            arrs = [get(k) for k in keys]
            for a in arrs:
                if not (hasattr(a, "is_cuda") and a.is_cuda and a.is_contiguous()
                        and str(a.dtype) == "torch.float32"):
                    raise TypeError("device phantom arrays must be contiguous float32 GPU tensors")
            goff = get("group_off")
            n = int(arrs[0].numel())
        else:
            arrs = [np.ascontiguousarray(get(k), dtype=np.float32) for k in keys]
            goff = phantom.group_off
            n = int(arrs[0].shape[0])
        for a in arrs[1:]:
            if (a.numel() if device else a.shape[0]) != n:
                raise ValueError("phantom arrays differ in length")
        self.keep += arrs
        # receive coils: [n_coils, n] sensitivities
        n_coils, sre, sim = 0, None, None
        if device and get("sens_re") is not None:
            sre, sim = get("sens_re"), get("sens_im")
            for a in (sre, sim):
                if not (a.is_cuda and a.is_contiguous() and str(a.dtype) == "torch.float32" and a.dim() == 2
                        and a.shape[1] == n):
                    raise TypeError("device sensitivities must be contiguous float32 GPU tensors [n_coils, n]")
            n_coils = int(sre.shape[0])
        elif not device and get("sens") is not None:
            sens = np.asarray(get("sens"))
            if sens.ndim != 2 or sens.shape[1] != n:
                raise ValueError("sensitivities must be [n_coils, n]")
            sre = np.ascontiguousarray(sens.real, dtype=np.float32)
            sim = np.ascontiguousarray(sens.imag, dtype=np.float32)
            n_coils = int(sens.shape[0])
        if n_coils:
            self.keep += [sre, sim]
        self.n_coils = n_coils
        self.n_sig = max(n_coils, 1)
        if goff is not None:
            goff = np.ascontiguousarray(goff, dtype=np.int64)
            self.keep.append(goff)
        ng = 1 if goff is None else int(goff.shape[0] - 1)
        self.n_groups = ng
        self.n = n
        self.c = koma_phantom(n, *[_ptr(a) for a in arrs[:7]], ng, _ptr(goff),
                              *([_ptr(a) for a in arrs[7:]] if moving else [None] * 3),
                              n_coils, _ptr(sre), _ptr(sim))


class _SeqArgs:
    def __init__(self, seq):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
        self.keep = [f64(seq.t), f64(seq.gx), f64(seq.gy), f64(seq.gz), f64(np.real(seq.b1)),
                     f64(np.imag(seq.b1)), np.ascontiguousarray(seq.adc_idx, dtype=np.int64)]
        k = self.keep
        self.n_adc = int(k[6].shape[0])
        self.c = koma_sequence(int(k[0].shape[0]), *[_ptr(a) for a in k[:6]], self.n_adc,
                               _ptr(k[6]) if self.n_adc else None)


class _BlockArgs:
    """koma_block array for a list of block descriptions (objects with
    ``duration``, ``gx``/``gy``/``gz`` (None, a trapezoid with amp / delay /
    rise / flat / fall, or a waveform with vertex arrays ``t`` and ``amp``),
    ``rf`` (None or delay / dt / complex ``samples``) and ``adc`` (None or
    delay / dwell / n))."""

    def __init__(self, blocks):
        self.keep = []
        n = len(blocks)
        self.n = n
        self.c = (koma_block * max(n, 1))()
        for i, b in enumerate(blocks):
            cb = self.c[i]
            cb.duration = float(b.duration)
            for a, g in enumerate((b.gx, b.gy, b.gz)):
                cg = cb.g[a]
                if g is None:
                    cg.kind = KOMA_GRAD_NONE
                elif hasattr(g, "rise"):
                    cg.kind = KOMA_GRAD_TRAP
                    cg.trap = koma_trap(float(g.amp), float(g.delay), float(g.rise), float(g.flat),
                                        float(g.fall))
                else:
                    tv = np.ascontiguousarray(g.t, dtype=np.float64)
                    av = np.ascontiguousarray(g.amp, dtype=np.float64)
                    self.keep += [tv, av]
                    cg.kind = KOMA_GRAD_PWL
                    cg.pwl_n = int(tv.shape[0]) if tv.shape == av.shape else -1
                    cg.pwl_t, cg.pwl_amp = _ptr(tv), _ptr(av)
            if b.rf is not None:
                smp = np.asarray(b.rf.samples, dtype=np.complex128)
                re = np.ascontiguousarray(smp.real)
                im = np.ascontiguousarray(smp.imag)
                self.keep += [re, im]
                cb.rf = koma_rf(float(b.rf.delay), float(b.rf.dt), int(smp.shape[0]), _ptr(re), _ptr(im))
            if b.adc is not None:
                cb.adc = koma_adc(float(b.adc.delay), float(b.adc.dwell), int(b.adc.n))


def koma_discretize(blocks, dt_max: float = np.inf, dt_rf_max: float = np.inf, name: str = "discretised"):
    """Sequence-aware discretisation of a block list (two calls: sizes, then
    values). Returns a sequence object with ``t``, ``gx``, ``gy``, ``gz``,
    complex ``b1`` per interval and ``adc_idx``."""
    from .workloads import Sequence
    b = _BlockArgs(blocks)
    L = lib()
    n_t, n_adc = c_int64(0), c_int64(0)
    _check(L.koma_discretize(b.c, b.n, float(dt_max), float(dt_rf_max), ctypes.byref(n_t),
                             ctypes.byref(n_adc), *([None] * 7)))
    t, gx, gy, gz = (np.empty(n_t.value) for _ in range(4))
    re, im = np.empty(max(n_t.value - 1, 0)), np.empty(max(n_t.value - 1, 0))
    adc = np.empty(n_adc.value, dtype=np.int64)
    _check(L.koma_discretize(b.c, b.n, float(dt_max), float(dt_rf_max), ctypes.byref(n_t),
                             ctypes.byref(n_adc), *[_ptr(a) for a in (t, gx, gy, gz, re, im)],
                             _ptr(adc) if n_adc.value else None))
    return Sequence(t, gx, gy, gz, re + 1j * im, adc, name=name,
                    meta={"dt_max": dt_max, "dt_rf_max": dt_rf_max, "n_blocks": b.n})


# ---------------------------------------------------------------- 1:1 wrappers
def koma_footprint(phantom, seq, cfg: koma_config) -> int:
    p, s = _PhantomArgs(phantom, False), _SeqArgs(seq)
    out = c_size_t(0)
    _check(lib().koma_footprint(ctypes.byref(p.c), ctypes.byref(s.c), ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def koma_plan_info(scanner, phantom, seq, cfg: koma_config, device: bool = False) -> dict:
    p, s = _PhantomArgs(phantom, device), _SeqArgs(seq)
    info = koma_req_info()
    sc = make_scanner(scanner)
    _check(lib().koma_plan_info(ctypes.byref(sc), ctypes.byref(p.c), ctypes.byref(s.c), ctypes.byref(cfg),
                                ctypes.byref(info)))
    return info.as_dict()


class Context:
    """A koma_ctx on one HIP device."""

    def __init__(self, device: int = 0, precision="mixed", **cfg):
        self.cfg = make_config(precision, **cfg)
        h = c_void_p()
        st = lib().koma_ctx_create(int(device), ctypes.byref(self.cfg), ctypes.byref(h))
        _check(st, None)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().koma_ctx_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def set_config(self, precision=None, **kw):
        c = koma_config.from_buffer_copy(self.cfg)
        if precision is not None:
            c.precision = {"fp64": KOMA_FP64, "mixed": KOMA_MIXED}[precision]
        for k, v in kw.items():
            setattr(c, k, v)
        _check(lib().koma_ctx_set_config(self.h, ctypes.byref(c)), self.h)
        self.cfg = c

    def simulate(self, scanner, phantom, seq, where: str = "host", stream=None, sig=None,
                 want_m: bool = False):
        """koma_simulate. ``where='host'``: numpy phantom, returns complex128
        ``[n_groups, n_adc]``, or ``[n_coils, n_groups, n_adc]`` for a phantom
        with coil sensitivities (and ``[n, 3]`` final M if ``want_m``).
        ``where='device'``: torch GPU tensors (dict or object with x..dw,
        optional vx, vy, vz and sens_re, sens_im; group_off on the host);
        ``sig`` a float64 GPU tensor ``[(n_coils,) n_groups, n_adc, 2]``
        that is written in place."""
        dev = where == "device"
        p, s = _PhantomArgs(phantom, dev), _SeqArgs(seq)
        sc = make_scanner(scanner)
        stream_h = None if stream is None else c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        if dev:
            if sig is None:
                raise ValueError("device simulate needs a preallocated sig tensor")
            if sig.numel() != 2 * p.n_sig * p.n_groups * s.n_adc or not sig.is_contiguous():
                raise ValueError("sig must be a contiguous [(n_coils,) n_groups, n_adc, 2] tensor")
            m = None
            if want_m:
                import torch
                m = torch.empty((p.n, 3), dtype=torch.float64, device=sig.device)
            _check(lib().koma_simulate(self.h, ctypes.byref(sc), ctypes.byref(p.c), ctypes.byref(s.c),
                                       KOMA_DEVICE, stream_h, _ptr(sig), _ptr(m)), self.h)
            return (sig, m) if want_m else sig
        out = np.zeros((p.n_sig, p.n_groups, s.n_adc, 2), dtype=np.float64)
        m = np.zeros((p.n, 3), dtype=np.float64) if want_m else None
        _check(lib().koma_simulate(self.h, ctypes.byref(sc), ctypes.byref(p.c), ctypes.byref(s.c),
                                   KOMA_HOST, stream_h, _ptr(out), _ptr(m)), self.h)
        z = out[..., 0] + 1j * out[..., 1]
        if not p.n_coils:
            z = z[0]
        return (z, m) if want_m else z

    def bind_async(self, scanner, phantom, seq, sig, stream=None, m_final=None, status=None,
                   noalloc: bool = False):
        """koma_simulate_async with its arguments marshalled once: returns a
        function of no arguments that enqueues one whole simulation (host
        packing included) on ``stream`` and returns without waiting. The
        phantom is device-resident (as for ``simulate(where='device')``),
        ``sig`` a float64 GPU tensor ``[(n_coils,) n_groups, n_adc, 2]``,
        ``m_final`` None or a float64 GPU tensor ``[n, 3]``, ``status`` None or
        an int32 GPU tensor of one element that receives the phantom's
        validation bits (0: valid; otherwise the outputs are left untouched).
        The tensors and arrays must stay alive until the work has run.
        ``noalloc``: koma_simulate_noalloc instead (the same work in the
        library's static device scratch, no allocation)."""
        p, s = _PhantomArgs(phantom, True), _SeqArgs(seq)
        sc = make_scanner(scanner)
        if sig.numel() != 2 * p.n_sig * p.n_groups * s.n_adc or not sig.is_contiguous():
            raise ValueError("sig must be a contiguous [(n_coils,) n_groups, n_adc, 2] tensor")
        if m_final is not None and (m_final.numel() != 3 * p.n or not m_final.is_contiguous()):
            raise ValueError("m_final must be a contiguous [n, 3] tensor")
        if status is not None and (status.numel() < 1 or str(status.dtype) != "torch.int32"):
            raise ValueError("status must be an int32 tensor")
        stream_h = None if stream is None else c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        args = (self.h, ctypes.byref(sc), ctypes.byref(p.c), ctypes.byref(s.c), stream_h, _ptr(sig),
                _ptr(m_final), _ptr(status))
        fn = lib().koma_simulate_noalloc if noalloc else lib().koma_simulate_async
        h = self.h
        keep = (p, s, sc, sig, m_final, status)

        def enqueue():
            _check(fn(*args), h)
            return keep[3]
        return enqueue

    def simulate_async(self, scanner, phantom, seq, sig, stream=None, m_final=None, status=None):
        """koma_simulate_async once (see ``bind_async``)."""
        return self.bind_async(scanner, phantom, seq, sig, stream, m_final, status)()

    def simulate_noalloc(self, scanner, phantom, seq, sig, stream=None, m_final=None, status=None):
        """koma_simulate_noalloc once: ``simulate_async`` without any device
        allocation (see ``bind_async``)."""
        return self.bind_async(scanner, phantom, seq, sig, stream, m_final, status, noalloc=True)()

    def mrf_match(self, dictionary, fingerprints, where: str = "host", stream=None, best=None, proj=None):
        """koma_mrf_match. Host: complex ``[n_entries, n_t]`` and ``[n_pix, n_t]``
        arrays (rounded to complex64), returns (best int32 [n_pix], proj complex128
        [n_pix]). Device: float32 GPU tensors ``[n, n_t, 2]`` and preallocated
        ``best`` (int32 [n_pix]) and ``proj`` (float64 [n_pix, 2]) tensors."""
        sh = None if stream is None else c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        if where == "device":
            for t in (dictionary, fingerprints):
                if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float32" and t.dim() == 3
                        and t.shape[2] == 2):
                    raise TypeError("device operands must be contiguous float32 GPU tensors [n, n_t, 2]")
            n_e, n_t = int(dictionary.shape[0]), int(dictionary.shape[1])
            n_p = int(fingerprints.shape[0])
            if int(fingerprints.shape[1]) != n_t or best is None or proj is None:
                raise ValueError("mismatched n_t or missing output tensors")
            if best.numel() != n_p or proj.numel() != 2 * n_p:
                raise ValueError("output tensors have the wrong size")
            _check(lib().koma_mrf_match(self.h, _ptr(dictionary), n_e, _ptr(fingerprints), n_p, n_t, KOMA_DEVICE,
                                        sh, _ptr(best), _ptr(proj)), self.h)
            return best, proj
        d = np.ascontiguousarray(np.asarray(dictionary, dtype=np.complex64))
        x = np.ascontiguousarray(np.asarray(fingerprints, dtype=np.complex64))
        if d.ndim != 2 or x.ndim != 2 or d.shape[1] != x.shape[1]:
            raise ValueError("dictionary [n_entries, n_t] and fingerprints [n_pix, n_t] expected")
        b = np.zeros(x.shape[0], dtype=np.int32)
        pr = np.zeros((x.shape[0], 2), dtype=np.float64)
        _check(lib().koma_mrf_match(self.h, _ptr(d), d.shape[0], _ptr(x), x.shape[0], d.shape[1], KOMA_HOST, sh,
                                    _ptr(b), _ptr(pr)), self.h)
        return b, pr[:, 0] + 1j * pr[:, 1]

    def mrf_svd(self, dictionary, rank: int = 5, oversample: int = 11, iters: int = 30):
        """koma_mrf_svd on a host dictionary ``[n_entries, n_t]``: returns
        (basis complex128 [n_t, rank], singular values [rank])."""
        d = np.ascontiguousarray(np.asarray(dictionary, dtype=np.complex64))
        n_e, n_t = d.shape
        basis = np.zeros((n_t, rank, 2), dtype=np.float64)
        sv = np.zeros(rank, dtype=np.float64)
        _check(lib().koma_mrf_svd(self.h, _ptr(d), n_e, n_t, int(rank), int(oversample), int(iters), KOMA_HOST, None,
                                  _ptr(basis), _ptr(sv)), self.h)
        return basis[..., 0] + 1j * basis[..., 1], sv

    def mrf_project(self, rows, basis):
        """koma_mrf_project on host arrays: coefficients complex64 [n_rows, rank]."""
        x = np.ascontiguousarray(np.asarray(rows, dtype=np.complex64))
        b = np.asarray(basis, dtype=np.complex128)
        bb = np.ascontiguousarray(np.stack([b.real, b.imag], -1))
        n_rows, n_t = x.shape
        rank = b.shape[1]
        if b.shape[0] != n_t:
            raise ValueError("basis must be [n_t, rank]")
        out = np.zeros((n_rows, rank), dtype=np.complex64)
        _check(lib().koma_mrf_project(self.h, _ptr(x), n_rows, n_t, _ptr(bb), rank, KOMA_HOST, None, _ptr(out)),
               self.h)
        return out

    def open(self, scanner, phantom, seq, where: str = "host") -> "Request":
        return Request(self, scanner, phantom, seq, where)

    def mem(self) -> dict:
        """koma_ctx_mem: device bytes held by open requests, cached for reuse,
        and the peak of their sum."""
        h, c, p = c_size_t(0), c_size_t(0), c_size_t(0)
        _check(lib().koma_ctx_mem(self.h, ctypes.byref(h), ctypes.byref(c), ctypes.byref(p)), self.h)
        return {"held": h.value, "cached": c.value, "peak": p.value}

    def profile(self, on: bool = True):
        _check(lib().koma_ctx_profile(self.h, 1 if on else 0), self.h)

    def kernel_stats(self, kind) -> dict:
        k = KERNEL_KINDS[kind] if isinstance(kind, str) else int(kind)
        ms, n, w = c_double(0), c_int64(0), c_int64(0)
        _check(lib().koma_ctx_kernel_stats(self.h, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(w)), self.h)
        return {"total_ms": ms.value, "launches": n.value, "work": w.value}


class Request:
    """A koma_req: phantom and spin state resident on the device."""

    def __init__(self, ctx: Context, scanner, phantom, seq, where="host"):
        self.ctx = ctx
        p, s = _PhantomArgs(phantom, where == "device"), _SeqArgs(seq)
        sc = make_scanner(scanner)
        h = c_void_p()
        _check(lib().koma_req_open(ctx.h, ctypes.byref(sc), ctypes.byref(p.c), ctypes.byref(s.c),
                                   KOMA_DEVICE if where == "device" else KOMA_HOST, ctypes.byref(h)), ctx.h)
        self.h = h
        self.n_groups, self.n_adc, self.n_coils = p.n_groups, s.n_adc, p.n_coils

    def advance(self, max_events: int = 0, stream=None):
        sh = None if stream is None else c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        _check(lib().koma_req_advance(self.h, int(max_events), sh), self.ctx.h)

    def done(self) -> bool:
        d = c_int(0)
        _check(lib().koma_req_done(self.h, ctypes.byref(d)), self.ctx.h)
        return bool(d.value)

    def result(self, stream=None) -> np.ndarray:
        sh = None if stream is None else c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        out = np.zeros((max(self.n_coils, 1), self.n_groups, self.n_adc, 2), dtype=np.float64)
        _check(lib().koma_req_result(self.h, _ptr(out), sh), self.ctx.h)
        z = out[..., 0] + 1j * out[..., 1]
        return z if self.n_coils else z[0]

    def save(self) -> bytes:
        n = c_size_t(0)
        _check(lib().koma_req_save(self.h, None, ctypes.byref(n)), self.ctx.h)
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().koma_req_save(self.h, buf, ctypes.byref(n)), self.ctx.h)
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        _check(lib().koma_req_load(self.h, blob, len(blob)), self.ctx.h)

    def info(self) -> dict:
        i = koma_req_info()
        _check(lib().koma_req_info_get(self.h, ctypes.byref(i)), self.ctx.h)
        return i.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib().koma_req_close(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def device_phantom(phantom, device="cuda:0") -> dict:
    """Copy a workloads.Phantom into float32 GPU tensors (group offsets stay on the host)."""
    import torch
    keys = _PhantomArgs.KEYS + (_PhantomArgs.VEL if getattr(phantom, "vx", None) is not None else ())
    d = {k: torch.from_numpy(np.ascontiguousarray(getattr(phantom, k), dtype=np.float32)).to(device)
         for k in keys}
    d["group_off"] = phantom.group_off
    if getattr(phantom, "sens", None) is not None:
        d["sens_re"] = torch.from_numpy(np.ascontiguousarray(phantom.sens.real, dtype=np.float32)).to(device)
        d["sens_im"] = torch.from_numpy(np.ascontiguousarray(phantom.sens.imag, dtype=np.float32)).to(device)
    return d
