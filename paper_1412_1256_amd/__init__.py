"""MI355X-native spectrometer path of PolariS (Mizuno et al., arXiv 1412.1256): Python binding.

The compute runs in ``libpolaris.so`` (hand-written gfx950 HIP kernels behind the C ABI of
``include/polaris.h``).  This module only marshals arguments: torch provides device memory and the stream.
There is no fallback: importing the binding when the library is missing raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Sequence

__all__ = ["PolarisError", "Instance", "Plan", "unpack", "lib", "LIB_PATH", "WIN", "PREC", "ACC"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpolaris.so")

WIN = {"rect": 0, "hann": 1, "taps": 2, "hamming": 3, "blackman": 4}
PREC = {"fp32": 0, "fp16": 1, "bf16": 2}
ACC = {"fp64": 0, "kahan32": 1}

STATUS = {0: "PS_OK", 1: "PS_ERR_ARG", 2: "PS_ERR_SIZE", 3: "PS_ERR_UNSUPPORTED", 4: "PS_ERR_STATE",
          5: "PS_ERR_WORKSPACE", 6: "PS_ERR_HIP"}


class PolarisError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        self.code = STATUS.get(status, f"PS_{status}")
        super().__init__(f"{self.code}: {detail}")


class _Instance(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("n_pairs", C.c_int32), ("pair_x", C.c_int32 * 4),
                ("pair_y", C.c_int32 * 4), ("bits", C.c_int32), ("window", C.c_int32), ("n_taps", C.c_int32),
                ("precision", C.c_int32), ("accum", C.c_int32), ("chunk_frames", C.c_int32),
                ("fft_len", C.c_int64), ("sample_rate_hz", C.c_double), ("hop", C.c_int64)]


class _Cal(C.Structure):
    _fields_ = [("gain_x", C.c_void_p), ("gain_y", C.c_void_p), ("dterms", C.c_void_p), ("psi", C.c_double),
                ("feed", C.c_int32), ("reserved", C.c_int32)]


FEED = {"linear": 0, "circular": 1}


class _CalGrad(C.Structure):
    _fields_ = [("d_gain_x", C.c_void_p), ("d_gain_y", C.c_void_p), ("d_dterms", C.c_void_p),
                ("d_taps", C.c_void_p)]


class _Schedule(C.Structure):
    _fields_ = [("log2_n1", C.c_int32), ("colpass_cols", C.c_int32), ("rowpass_frames", C.c_int32),
                ("col_wg_per_cu", C.c_int32), ("rowpass_slots", C.c_int32), ("single_pass", C.c_int32)]


@dataclass(frozen=True)
class Schedule:
    """Pass schedule of one instance (see ``ps_schedule``); 0 = default."""
    log2_n1: int = 0
    colpass_cols: int = 0
    rowpass_frames: int = 0
    col_wg_per_cu: int = 0
    rowpass_slots: int = 0
    single_pass: int = 0  # 0 default, 1 whole frames in LDS (2^8 .. 2^12 points, FP32), 2 four-step passes

    def to_c(self) -> _Schedule:
        return _Schedule(self.log2_n1, self.colpass_cols, self.rowpass_frames, self.col_wg_per_cu,
                         self.rowpass_slots, self.single_pass)


def schedule_candidates(instance) -> list:
    """Every schedule the library can run the instance with."""
    c = instance.to_c()
    n = C.c_int32()
    _check(lib().ps_schedule_candidates(C.byref(c), None, 0, C.byref(n)))
    arr = (_Schedule * max(1, n.value))()
    _check(lib().ps_schedule_candidates(C.byref(c), arr, n.value, C.byref(n)))
    return [Schedule(a.log2_n1, a.colpass_cols, a.rowpass_frames, a.col_wg_per_cu, a.rowpass_slots, a.single_pass)
            for a in arr[:n.value]]


_LIB = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "ps_plan": [C.POINTER(_Instance), i32, C.POINTER(vp), C.POINTER(sz)],
            "ps_bind": [vp, vp, sz, vp],
            "ps_set_window_taps": [vp, i32, vp],
            "ps_reset": [vp],
            "ps_accumulate": [vp, C.POINTER(vp), C.POINTER(i64)],
            "ps_spectra": [vp, i32, vp, C.POINTER(i64)],
            "ps_stokes": [vp, i32, C.POINTER(_Cal), vp],
            "ps_calibrate_backward": [vp, i32, vp, i64, C.POINTER(_Cal), vp, C.POINTER(_CalGrad)],
            "ps_state_bytes": [vp, i32, C.POINTER(sz)],
            "ps_state_export": [vp, i32, vp, C.POINTER(i64)],
            "ps_state_import": [vp, i32, vp, i64],
            "ps_unpack": [vp, i32, i32, i64, vp, vp],
            "ps_destroy": [vp],
            "ps_status_string": [C.c_int],
            "ps_last_error": [],
            "ps_version": [],
            "ps_profile_enable": [vp, i32],
            "ps_profile_read": [vp, C.POINTER(C.c_double), C.POINTER(i64)],
            "ps_stokes_all": [vp, C.POINTER(_Cal), C.POINTER(vp)],
            "ps_accumulate_stokes": [vp, C.POINTER(vp), C.POINTER(i64), C.POINTER(_Cal), C.POINTER(vp)],
            "ps_plan_scheduled": [C.POINTER(_Instance), C.POINTER(_Schedule), i32, C.POINTER(vp), C.POINTER(sz)],
            "ps_schedule_candidates": [C.POINTER(_Instance), C.POINTER(_Schedule), i32, C.POINTER(i32)],
            "ps_set_histograms": [vp, i32, i32],
            "ps_histograms": [vp, i32, vp, vp, C.POINTER(i64)],
            "ps_graph_begin": [vp],
            "ps_graph_end": [vp, i32],
            "ps_graph_launch": [vp],
            "ps_channel_average": [vp, i64, i64, i32, vp, vp, vp, vp],
            "ps_bandpass_work_bytes": [i64, i32, C.c_double, C.POINTER(sz)],
            "ps_bandpass_fit": [vp, i64, i32, C.c_double, vp, sz, vp, vp],
            "ps_bandpass_correct": [vp, i64, i64, vp, vp, vp, vp],
            "ps_bandpass_fit_static": [vp, i64, i32, C.c_double, vp, vp],
            "ps_integration_id": [vp, i32, C.POINTER(C.c_uint64)],
            "ps_band_stats": [vp, i64, i64, vp, vp],
            "ps_allan_work_bytes": [i64, i64, i64, i64, i32, C.POINTER(sz)],
            "ps_allan": [vp, i64, i64, i64, i64, C.POINTER(i32), i32, C.c_double, i32, vp, sz, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.ps_status_string.restype = C.c_char_p
        L.ps_last_error.restype = C.c_char_p
        L.ps_version.restype = C.c_int32
        _LIB = L
    return _LIB


def _check(status: int):
    if status != 0:
        raise PolarisError(status, lib().ps_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclass
class Instance:
    """One sampler stream set (see ``ps_instance`` in include/polaris.h)."""
    fft_len: int
    bits: int = 8
    n_streams: int = 2
    pairs: Sequence[tuple] = ((0, 1),)
    window: str = "rect"
    n_taps: int = 0
    precision: str = "fp32"
    accum: str = "fp64"
    chunk_frames: int = 0
    sample_rate_hz: float = 16e6
    hop: int = 0  # samples between frame starts: 0 or fft_len (contiguous), fft_len / 2 (50 % overlap), / 4, / 8

    def to_c(self) -> _Instance:
        s = _Instance()
        s.n_streams = self.n_streams
        s.n_pairs = len(self.pairs)
        for i, (x, y) in enumerate(self.pairs[:4]):
            s.pair_x[i] = x
            s.pair_y[i] = y
        s.bits = self.bits
        s.window = WIN[self.window] if isinstance(self.window, str) else int(self.window)
        s.n_taps = self.n_taps
        s.precision = PREC[self.precision] if isinstance(self.precision, str) else int(self.precision)
        s.accum = ACC[self.accum] if isinstance(self.accum, str) else int(self.accum)
        s.chunk_frames = self.chunk_frames
        s.fft_len = self.fft_len
        s.sample_rate_hz = self.sample_rate_hz
        s.hop = self.hop
        return s

    @property
    def n_pairs(self):
        return len(self.pairs)

    @property
    def channels(self):
        return self.fft_len // 2

    @staticmethod
    def from_synth(d: dict, **over) -> "Instance":
        kw = dict(fft_len=d["fft_len"], bits=d["bits"], n_streams=d["n_streams"], pairs=tuple(d["pairs"]),
                  window=d["window"], n_taps=64 if d["window"] == "taps" else 0, hop=d.get("hop", 0))
        kw.update(over)
        return Instance(**kw)


def plan_workspace_bytes(instances: Sequence[Instance]) -> int:
    arr = (_Instance * len(instances))(*[i.to_c() for i in instances])
    h = C.c_void_p()
    nbytes = C.c_size_t()
    _check(lib().ps_plan(arr, len(instances), C.byref(h), C.byref(nbytes)))
    lib().ps_destroy(h)
    return nbytes.value


class Plan:
    """A bound plan: host metadata in the library, workspace in a torch uint8 tensor on one device."""

    def __init__(self, instances: Sequence[Instance], device=None, stream=None, schedules=None, tune: bool = False):
        """schedules: None or one Schedule (or None) per instance; tune=True takes each instance's schedule
        from the autotuner (its JSON cache, timing the candidates on this device on a miss)."""
        import torch
        self.torch = torch
        self.instances = list(instances)
        self.device = torch.device(device if device is not None else "cuda")
        if tune:
            from . import autotune
            schedules = [autotune.best_schedule(i, device=self.device) for i in self.instances]
        arr = (_Instance * len(self.instances))(*[i.to_c() for i in self.instances])
        h = C.c_void_p()
        nbytes = C.c_size_t()
        if schedules is None:
            _check(lib().ps_plan(arr, len(self.instances), C.byref(h), C.byref(nbytes)))
        else:
            if len(schedules) != len(self.instances):
                raise ValueError("one schedule per instance")
            sarr = (_Schedule * len(self.instances))(*[(x or Schedule()).to_c() for x in schedules])
            _check(lib().ps_plan_scheduled(arr, sarr, len(self.instances), C.byref(h), C.byref(nbytes)))
        self.schedules = schedules
        self._h = h
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # the library needs 256-byte alignment; over-allocate and offset
        self._ws_raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws_raw.data_ptr()) % 256
        self.workspace = self._ws_raw[off:off + nbytes.value]
        self.workspace_bytes = nbytes.value
        _check(lib().ps_bind(self._h, C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                             C.c_void_p(self.stream.cuda_stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.ps_destroy(h)
            self._h = None

    # --------------------------------------------------------------------------------------------
    def reset(self):
        _check(lib().ps_reset(self._h))

    def accumulate(self, packed, n_samples=None):
        """packed: one uint8 device tensor per instance (or a single tensor for a one-instance plan)."""
        if not isinstance(packed, (list, tuple)):
            packed = [packed]
        n = len(self.instances)
        if len(packed) != n:
            raise ValueError(f"expected {n} packed buffers, got {len(packed)}")
        ptrs = (C.c_void_p * n)(*[None if p is None else p.data_ptr() for p in packed])
        if n_samples is None:
            n_samples = []
            for inst, p in zip(self.instances, packed):
                bits_per_t = inst.n_streams * inst.bits
                n_samples.append(0 if p is None else p.numel() * 8 // bits_per_t)
        ns = (C.c_int64 * n)(*n_samples)
        _check(lib().ps_accumulate(self._h, ptrs, ns))

    def accumulate_stokes(self, packed, n_samples=None, outs=None, cals=None, gain_x=None, gain_y=None,
                          dterms=None, psi: float = 0.0, feed="linear", out=None):
        """accumulate() and then the Stokes spectra of every instance (ps_accumulate_stokes).  For a
        one-instance plan the calibration may be given as keywords and the output as out=; otherwise outs
        and cals as in stokes_all().  Returns the list of output tensors."""
        torch = self.torch
        if not isinstance(packed, (list, tuple)):
            packed = [packed]
        n = len(self.instances)
        if len(packed) != n:
            raise ValueError(f"expected {n} packed buffers, got {len(packed)}")
        ptrs = (C.c_void_p * n)(*[None if p is None else p.data_ptr() for p in packed])
        if n_samples is None:
            n_samples = [0 if p is None else p.numel() * 8 // (inst.n_streams * inst.bits)
                         for inst, p in zip(self.instances, packed)]
        ns = (C.c_int64 * n)(*n_samples)
        if outs is None:
            outs = [out] if (n == 1 and out is not None) else [
                torch.empty((I.n_pairs, 4, I.channels), dtype=torch.float32, device=self.device)
                for I in self.instances]
        optr = (C.c_void_p * n)(*[None if o is None else o.data_ptr() for o in outs])
        if cals is None and n == 1:
            cals = [(gain_x, gain_y, dterms, psi, feed)]
        arr, keep = None, []
        if cals is not None:
            arr = (_Cal * n)()
            for i, c in enumerate(cals):
                c = tuple(c) if c is not None else (None, None, None, 0.0)
                gx, gy, dt, ps_ = c[:4]
                fd = c[4] if len(c) > 4 else "linear"
                gx, gy, dt = self._as_f32(gx), self._as_f32(gy), self._as_f32(dt)
                keep += [gx, gy, dt]
                arr[i] = self._cal(gx, gy, dt, ps_, fd)
        self._cal_keepalive = keep
        _check(lib().ps_accumulate_stokes(self._h, ptrs, ns, arr, optr))
        return outs

    def spectra(self, inst: int = 0, out=None):
        I = self.instances[inst]
        if out is None:
            out = self.torch.empty((I.n_pairs, 4, I.channels), dtype=self.torch.float64, device=self.device)
        nf = C.c_int64()
        _check(lib().ps_spectra(self._h, inst, _ptr(out), C.byref(nf)))
        return out, nf.value

    def _cal(self, gain_x, gain_y, dterms, psi, feed="linear"):
        cal = _Cal()
        cal.gain_x = None if gain_x is None else gain_x.data_ptr()
        cal.gain_y = None if gain_y is None else gain_y.data_ptr()
        cal.dterms = None if dterms is None else dterms.data_ptr()
        cal.psi = float(psi)
        cal.feed = FEED[feed] if isinstance(feed, str) else int(feed)
        return cal

    def stokes(self, inst: int = 0, gain_x=None, gain_y=None, dterms=None, psi: float = 0.0, out=None,
               feed="linear"):
        """Calibrated I, Q, U, V [n_pairs][4][C] float32.  gains: float32 [P][C][2] (or complex64 [P][C]).
        feed: "linear" (Eq. 2, pair = X, Y) or "circular" (pair = R, L)."""
        I = self.instances[inst]
        gain_x, gain_y, dterms = (self._as_f32(gain_x), self._as_f32(gain_y), self._as_f32(dterms))
        if out is None:
            out = self.torch.empty((I.n_pairs, 4, I.channels), dtype=self.torch.float32, device=self.device)
        cal = self._cal(gain_x, gain_y, dterms, psi, feed)
        _check(lib().ps_stokes(self._h, inst, C.byref(cal), _ptr(out)))
        return out

    def stokes_all(self, outs=None, cals=None):
        """Stokes of every instance in one grouped launch.  outs: list of float32 [P][4][C] tensors (None
        entries skip an instance; default: new tensors); cals: None or a list of (gain_x, gain_y, dterms, psi)
        tuples (entries may be None)."""
        n = len(self.instances)
        if outs is None:
            outs = [self.torch.empty((I.n_pairs, 4, I.channels), dtype=self.torch.float32, device=self.device)
                    for I in self.instances]
        ptrs = (C.c_void_p * n)(*[None if o is None else o.data_ptr() for o in outs])
        calp = None
        if cals is not None:
            arr = (_Cal * n)()
            keep = []
            for i, c in enumerate(cals):
                gx, gy, dt, psi = c if c is not None else (None, None, None, 0.0)
                gx, gy, dt = self._as_f32(gx), self._as_f32(gy), self._as_f32(dt)
                keep += [gx, gy, dt]
                arr[i] = self._cal(gx, gy, dt, psi)
            self._cal_keepalive = keep
            calp = arr
        _check(lib().ps_stokes_all(self._h, calp, ptrs))
        return outs

    def set_histograms(self, on: bool = True, inst: int = 0):
        """Count the level histograms of instance inst's streams from the next integration on."""
        _check(lib().ps_set_histograms(self._h, inst, 1 if on else 0))

    def histograms(self, inst: int = 0):
        """(counts int64 [P][2][2^bits], power float64 [P][2][2], frames counted) of the current integration:
        power = (mean square level, sigma / threshold for 2-bit samplers or NaN)."""
        I = self.instances[inst]
        torch = self.torch
        counts = torch.empty((I.n_pairs, 2, 1 << I.bits), dtype=torch.int64, device=self.device)
        power = torch.empty((I.n_pairs, 2, 2), dtype=torch.float64, device=self.device)
        nf = C.c_int64()
        _check(lib().ps_histograms(self._h, inst, _ptr(counts), _ptr(power), C.byref(nf)))
        return counts, power, nf.value

    # --------------------------------------------------------------------------------------------
    # hipGraph capture of a whole integration (the plan must be bound to a non-default stream)
    def graph_capture(self, fn):
        """Run fn() once eagerly (puts the launch descriptors in place), then capture fn() into a graph."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            fn()
        _check(lib().ps_graph_begin(self._h))
        try:
            with torch.cuda.stream(self.stream):
                fn()
        except BaseException:
            lib().ps_graph_end(self._h, 0)  # discard the partial capture
            raise
        _check(lib().ps_graph_end(self._h, 1))

    def graph_replay(self):
        _check(lib().ps_graph_launch(self._h))

    def calibrate_backward(self, packed, dL_diquv, inst: int = 0, gain_x=None, gain_y=None, dterms=None,
                           psi: float = 0.0, want=("gain_x", "gain_y", "dterms", "taps")):
        I = self.instances[inst]
        torch = self.torch
        gain_x, gain_y, dterms = (self._as_f32(gain_x), self._as_f32(gain_y), self._as_f32(dterms))
        P, Cn = I.n_pairs, I.channels
        outs = {}
        grad = _CalGrad()
        if "gain_x" in want:
            outs["gain_x"] = torch.empty((P, Cn, 2), dtype=torch.float32, device=self.device)
            grad.d_gain_x = outs["gain_x"].data_ptr()
        if "gain_y" in want:
            outs["gain_y"] = torch.empty((P, Cn, 2), dtype=torch.float32, device=self.device)
            grad.d_gain_y = outs["gain_y"].data_ptr()
        if "dterms" in want:
            outs["dterms"] = torch.empty((P, 4), dtype=torch.float32, device=self.device)
            grad.d_dterms = outs["dterms"].data_ptr()
        if "taps" in want and I.window == "taps":
            outs["taps"] = torch.empty((I.n_taps,), dtype=torch.float32, device=self.device)
            grad.d_taps = outs["taps"].data_ptr()
        cal = self._cal(gain_x, gain_y, dterms, psi)
        n_samples = packed.numel() * 8 // (I.n_streams * I.bits)
        g = dL_diquv.to(torch.float32).contiguous()
        _check(lib().ps_calibrate_backward(self._h, inst, _ptr(packed), n_samples, C.byref(cal), _ptr(g),
                                           C.byref(grad)))
        return outs

    def integration_id(self, inst: int = 0) -> int:
        """Changes whenever the integration a gradient would be taken of changes (see ps_integration_id)."""
        v = C.c_uint64()
        _check(lib().ps_integration_id(self._h, inst, C.byref(v)))
        return v.value

    def set_window_taps(self, taps, inst: int = 0):
        t = self._as_f32(taps)
        n = self.instances[inst].n_taps
        if n > 0 and t.numel() != n:  # (an instance without a taps window is refused by the library)
            raise ValueError(f"instance {inst} has {n} window taps, got {t.numel()}")
        _check(lib().ps_set_window_taps(self._h, inst, _ptr(t)))
        self._taps_keepalive = t

    def state_bytes(self, inst: int = 0) -> int:
        n = C.c_size_t()
        _check(lib().ps_state_bytes(self._h, inst, C.byref(n)))
        return n.value

    def state_export(self, inst: int = 0):
        buf = self.torch.empty(self.state_bytes(inst), dtype=self.torch.uint8, device=self.device)
        nf = C.c_int64()
        _check(lib().ps_state_export(self._h, inst, _ptr(buf), C.byref(nf)))
        return buf, nf.value

    def state_import(self, buf, n_frames: int, inst: int = 0):
        _check(lib().ps_state_import(self._h, inst, _ptr(buf), int(n_frames)))

    KERNELS = ("colpass", "rowpass", "stokes", "spectra", "backward", "other")

    def profile_enable(self, on: bool = True):
        """Bracket every kernel this plan launches with hipEvents on its stream (measurement only)."""
        _check(lib().ps_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kernel: (total_ms, launches)} since the last read; waits for the recorded events."""
        ms = (C.c_double * 8)()
        n = (C.c_int64 * 8)()
        _check(lib().ps_profile_read(self._h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(self.KERNELS) if n[i]}

    def _as_f32(self, t):
        if t is None:
            return None
        torch = self.torch
        if t.is_complex():
            t = torch.view_as_real(t.to(torch.complex64))
        return t.to(device=self.device, dtype=torch.float32).contiguous()


def unpack(packed, bits: int, n_streams: int, n_time: int, stream=None):
    """Stand-alone data translation: float32 [n_streams][n_time] levels of a packed device buffer."""
    import torch
    out = torch.empty((n_streams, n_time), dtype=torch.float32, device=packed.device)
    s = stream if stream is not None else torch.cuda.current_stream(packed.device)
    _check(lib().ps_unpack(_ptr(packed), bits, n_streams, n_time, _ptr(out), C.c_void_p(s.cuda_stream)))
    return out


# ------------------------------------------------------------------------------------------------
# post-integration reductions (device tensors in, device tensors out; enqueued on the current stream)

def _stream(t, stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(t.device)
    return C.c_void_p(s.cuda_stream)


def _f32_2d(x):
    x = x.contiguous()
    if x.dtype != __import__("torch").float32:
        raise TypeError("float32 spectra expected")
    return x if x.dim() == 2 else x.reshape(-1, x.shape[-1])


def channel_average(spectra, factor: int, flags=None, stream=None):
    """Bins of `factor` channels along the last axis, flagged (uint8 [C], nonzero) and non-finite channels
    left out: (mean [..., C/factor] float32, counts [..., C/factor] int32)."""
    import torch
    x = _f32_2d(spectra)
    n_spec, n_chan = x.shape
    out = torch.empty((n_spec, n_chan // max(1, factor)), dtype=torch.float32, device=x.device)
    cnt = torch.empty(out.shape, dtype=torch.int32, device=x.device)
    fl = None if flags is None else flags.to(torch.uint8).contiguous()
    _check(lib().ps_channel_average(_ptr(x), n_spec, n_chan, factor, _ptr(fl), _ptr(out), _ptr(cnt),
                                    _stream(x, stream)))
    shape = tuple(spectra.shape[:-1]) + (out.shape[-1],)
    return out.reshape(shape), cnt.reshape(shape)


def bandpass_fit(h, knot_spacing: int = 128, edge_frac: float = 0.06, stream=None):
    """Smoothed bandpass: least-squares cubic spline with knots every knot_spacing channels, fitted without
    edge_frac of the band at each end (NaN there); float32 [C]."""
    import torch
    h = h.contiguous().to(torch.float32)
    n = C.c_size_t()
    _check(lib().ps_bandpass_work_bytes(h.numel(), knot_spacing, edge_frac, C.byref(n)))
    work = torch.empty(n.value + 256, dtype=torch.uint8, device=h.device)
    off = (-work.data_ptr()) % 256
    w = work[off:off + n.value]
    out = torch.empty_like(h)
    _check(lib().ps_bandpass_fit(_ptr(h), h.numel(), knot_spacing, edge_frac, _ptr(w), n.value, _ptr(out),
                                 _stream(h, stream)))
    out._work_keepalive = work
    return out


def bandpass_correct(hk, smooth, gain=None, stream=None):
    """H^_k = H_k / (G_k H): hk [n][C] float32, smooth [C] float32, gain [n] float64 or None."""
    import torch
    x = _f32_2d(hk)
    g = None if gain is None else gain.to(torch.float64).contiguous()
    out = torch.empty_like(x)
    _check(lib().ps_bandpass_correct(_ptr(x), x.shape[0], x.shape[1], _ptr(smooth.contiguous()), _ptr(g), _ptr(out),
                                     _stream(x, stream)))
    return out.reshape(hk.shape)


def band_stats(x, stream=None):
    """[n][2] float64: mean and standard deviation of each spectrum's finite channels."""
    import torch
    v = _f32_2d(x)
    out = torch.empty((v.shape[0], 2), dtype=torch.float64, device=v.device)
    _check(lib().ps_band_stats(_ptr(v), v.shape[0], v.shape[1], _ptr(out), _stream(v, stream)))
    return out


def allan(x, lags, spacing: float = 1.0, normalize: bool = False, axis: int = -1, stream=None):
    """Eq. 3 / Eq. 4 along `axis` of a 2-D float32 tensor (the other axis indexes the series): float64
    [n_series][len(lags)]."""
    import torch
    if x.dim() != 2:
        raise ValueError("a 2-D tensor expected")
    v = x.contiguous().to(torch.float32)
    axis = axis % 2
    n_points, n_series = v.shape[axis], v.shape[1 - axis]
    point_stride, series_stride = (1, n_points) if axis == 1 else (n_series, 1)
    lg = (C.c_int32 * len(lags))(*[int(L) for L in lags])
    out = torch.empty((n_series, len(lags)), dtype=torch.float64, device=v.device)
    nb = C.c_size_t()
    _check(lib().ps_allan_work_bytes(n_points, point_stride, n_series, series_stride, len(lags), C.byref(nb)))
    work = torch.empty(max(8, nb.value), dtype=torch.uint8, device=v.device)
    _check(lib().ps_allan(_ptr(v), n_points, point_stride, n_series, series_stride, lg, len(lags), spacing,
                          1 if normalize else 0, _ptr(work), nb.value, _ptr(out), _stream(v, stream)))
    out._work_keepalive = work
    return out
