"""FP64 CPU oracle of the PolariS spectrometer path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.  It wraps
``liboracle.so`` (plain C, FP64, built from ``polaris_oracle.c`` by ``oracle/build.py``) with numpy
conveniences.  Array conventions follow the C header: raw products ``acc[p][q][k]`` with
q = XX*, YY*, Re XY*, Im XY*; Stokes ``iquv[p][0..3][k]``; complex parameters as complex128 arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

WIN = {"rect": 0, "hann": 1, "taps": 2, "hamming": 3, "blackman": 4}


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        src = os.path.join(HERE, "polaris_oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            from . import build as _b
            _b.build()
        lib = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        u8 = C.POINTER(C.c_uint8)
        ip = C.POINTER(C.c_int)
        i64 = C.c_int64
        lib.or_unpack.argtypes = [u8, C.c_int, C.c_int, i64, dp]
        lib.or_window.argtypes = [C.c_int, i64, dp, C.c_int, dp, dp]
        lib.or_fft.argtypes = [dp, dp, i64]
        lib.or_dft.argtypes = [dp, dp, i64, dp, dp]
        lib.or_accumulate.argtypes = [u8, C.c_int, C.c_int, i64, i64, i64, dp, C.c_int, ip, ip, C.c_int, dp,
                                      C.POINTER(i64)]
        lib.or_stokes.argtypes = [dp, C.c_int, i64, i64, C.c_double, dp, dp, dp, C.c_double, C.c_int, dp]
        lib.or_calibrate_backward.argtypes = [u8, C.c_int, C.c_int, i64, i64, i64, dp, dp, C.c_int, C.c_int, ip, ip,
                                              dp, i64, C.c_double, dp, dp, dp, C.c_double, dp, C.c_int,
                                              dp, dp, dp, dp, dp]
        for f in ("or_unpack", "or_window", "or_fft", "or_dft", "or_accumulate", "or_stokes",
                  "or_calibrate_backward"):
            getattr(lib, f).restype = C.c_int
        _LIB = lib
    return _LIB


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _cplx_arg(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(shape))
    return a.view(np.float64)


# ------------------------------------------------------------------------------------------------

def unpack(packed, bits: int, n_streams: int, n_time: int) -> np.ndarray:
    packed = np.ascontiguousarray(packed, dtype=np.uint8)
    out = np.empty((n_streams, n_time), dtype=np.float64)
    _check(_lib().or_unpack(_u8(packed), bits, n_streams, n_time, _dp(out)), "unpack")
    return out


def window(kind: str, n: int, taps=None):
    w = np.empty(n, dtype=np.float64)
    s = C.c_double(0.0)
    t = None if taps is None else np.ascontiguousarray(taps, dtype=np.float64)
    _check(_lib().or_window(WIN[kind], n, _dp(t), 0 if t is None else t.size, _dp(w), C.byref(s)), "window")
    return w, s.value


def fft(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    _check(_lib().or_fft(_dp(re), _dp(im), x.size), "fft")
    return re + 1j * im


def dft(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    ore = np.empty_like(re)
    oim = np.empty_like(im)
    _check(_lib().or_dft(_dp(re), _dp(im), x.size, _dp(ore), _dp(oim)), "dft")
    return ore + 1j * oim


def _pairs(pairs):
    px = np.ascontiguousarray([p[0] for p in pairs], dtype=np.int32)
    py = np.ascontiguousarray([p[1] for p in pairs], dtype=np.int32)
    return px, py


def accumulate(packed, bits, n_streams, n_time, fft_len, w, pairs, nthreads=0, hop=0):
    """Raw products acc[p][4][C] and the frame count; frame f starts at sample f * hop (0: fft_len)."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.float64)
    px, py = _pairs(pairs)
    C_ = fft_len // 2
    acc = np.empty((len(pairs), 4, C_), dtype=np.float64)
    nf = C.c_int64(0)
    ip = C.POINTER(C.c_int)
    _check(_lib().or_accumulate(_u8(packed), bits, n_streams, n_time, fft_len, hop, _dp(w), len(pairs),
                                px.ctypes.data_as(ip), py.ctypes.data_as(ip), nthreads, _dp(acc), C.byref(nf)),
           "accumulate")
    return acc, nf.value


def stokes(acc, n_frames, sumw2, gain_x=None, gain_y=None, dterms=None, psi=0.0, feed="linear"):
    """Eq. 2 (linear feeds) or the circular-feed combination (streams R, L) of the calibrated coherency."""
    acc = np.ascontiguousarray(acc, dtype=np.float64)
    P, _, C_ = acc.shape
    gx = _cplx_arg(gain_x, (P, C_))
    gy = _cplx_arg(gain_y, (P, C_))
    dt = _cplx_arg(dterms, (P, 2))
    out = np.empty((P, 4, C_), dtype=np.float64)
    f = {"linear": 0, "circular": 1}[feed]
    _check(_lib().or_stokes(_dp(acc), P, C_, n_frames, sumw2, _dp(gx), _dp(gy), _dp(dt), psi, f, _dp(out)),
           "stokes")
    return out


def calibrate_backward(packed, bits, n_streams, n_time, fft_len, w, pairs, acc, n_frames, sumw2, g_iquv,
                       gain_x=None, gain_y=None, dterms=None, psi=0.0, taps=None, nthreads=0, hop=0):
    """Returns dict with d_gain_x, d_gain_y ([P][C] complex), d_dterms ([P][2] complex), d_w, d_taps."""
    packed = np.ascontiguousarray(packed, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.float64)
    acc = np.ascontiguousarray(acc, dtype=np.float64)
    P, _, C_ = acc.shape
    px, py = _pairs(pairs)
    gx = _cplx_arg(gain_x, (P, C_))
    gy = _cplx_arg(gain_y, (P, C_))
    dt = _cplx_arg(dterms, (P, 2))
    g = np.ascontiguousarray(g_iquv, dtype=np.float64)
    t = None if taps is None else np.ascontiguousarray(taps, dtype=np.float64)
    dgx = np.zeros((P, C_, 2))
    dgy = np.zeros((P, C_, 2))
    ddt = np.zeros((P, 4))
    dw = np.zeros(fft_len)
    dtaps = np.zeros(0 if t is None else t.size)
    ip = C.POINTER(C.c_int)
    _check(_lib().or_calibrate_backward(
        _u8(packed), bits, n_streams, n_time, fft_len, hop, _dp(w), _dp(t), 0 if t is None else t.size, P,
        px.ctypes.data_as(ip), py.ctypes.data_as(ip), _dp(acc), n_frames, sumw2, _dp(gx), _dp(gy), _dp(dt), psi,
        _dp(g), nthreads, _dp(dgx), _dp(dgy), _dp(ddt), _dp(dw), _dp(dtaps) if t is not None else None),
        "calibrate_backward")
    return dict(d_gain_x=dgx[..., 0] + 1j * dgx[..., 1], d_gain_y=dgy[..., 0] + 1j * dgy[..., 1],
                d_dterms=(ddt[:, 0::2] + 1j * ddt[:, 1::2]), d_w=dw, d_taps=dtaps)


def run_instance(inst: dict, taps=None, nthreads: int = 0):
    """Raw products, frame count and window sum of squares of a synth instance dict."""
    w, s2 = window(inst["window"], inst["fft_len"], taps=taps)
    acc, nf = accumulate(inst["packed"], inst["bits"], inst["n_streams"], inst["n_samples"], inst["fft_len"], w,
                         inst["pairs"], nthreads=nthreads, hop=inst.get("hop", 0))
    return acc, nf, s2, w


# ------------------------------------------------------------------------------------------------
# level histograms and total power (Sec. 2: total power from the samplers' bit distributions)

def level_histograms(packed, bits: int, n_streams: int, n_time: int, pairs) -> np.ndarray:
    """Counts [P][2 (X, Y)][2^bits] of every sample of each pair's streams, bins in ascending level order.
    Plain definition: decode every item (the pinned unpack) and count equal levels.  (With overlapped
    frames every sample is counted once, as it leaves the segmentation: pass the samples up to the last
    N - hop of the stream, which are counted with the next call's data.)"""
    levels = unpack(packed, bits, n_streams, n_time)
    nbin = 1 << bits
    lv = np.arange(nbin) - 128 if bits == 8 else 2 * np.arange(nbin) - (nbin - 1)
    out = np.zeros((len(pairs), 2, nbin), dtype=np.int64)
    for p, (x, y) in enumerate(pairs):
        for j, s in enumerate((x, y)):
            for b in range(nbin):
                out[p, j, b] = int(np.count_nonzero(levels[s] == lv[b]))
    return out


def total_power(counts: np.ndarray, bits: int) -> np.ndarray:
    """[P][2][2]: the mean square level, and for 2-bit samplers sigma / threshold from the fraction P of
    samples in the inner levels, P(|x| < theta) = erf(theta / (sigma sqrt 2)) (NaN for other formats)."""
    from scipy.special import erfinv
    nbin = 1 << bits
    lv = np.arange(nbin) - 128.0 if bits == 8 else 2.0 * np.arange(nbin) - (nbin - 1)
    P = counts.shape[0]
    out = np.full((P, 2, 2), np.nan)
    for p in range(P):
        for j in range(2):
            c = counts[p, j].astype(np.float64)
            n = c.sum()
            out[p, j, 0] = float((lv * lv * c).sum() / n) if n > 0 else 0.0
            if bits == 2 and n > 0:
                pin = (c[1] + c[2]) / n
                if 0.0 < pin < 1.0:
                    out[p, j, 1] = 1.0 / (np.sqrt(2.0) * erfinv(pin))
    return out
