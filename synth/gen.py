"""Seeded input generators (sampler emulation).

Wire layout produced here (the layout the spectrometer consumes):

* one byte buffer per instance, time-major and stream-interleaved: the code of
  time step t and stream s is item ``t*S + s``;
* b-bit codes (b = 2, 4, 8) sit at bit offset ``item*b``, least significant
  bits first inside each byte;
* b = 8 codes are two's-complement int8 samples;
* b = 32 items are little-endian IEEE float32 samples (test format).

Quantisers (the sampler's, not the spectrometer's):

* 2-bit: thresholds -theta, 0, +theta (theta = 1 sigma); code 0..3 counts how
  many thresholds the sample reaches (x >= threshold counts);
* 4-bit: uniform, step sigma/2, code = clip(floor(x/step) + 8, 0, 15);
* 8-bit: clip(rint(x), -128, 127) with x already in LSB units
  (sigma = 16 LSB by default), round half to even.

All randomness comes from ``numpy.random.PCG64`` seeded from
``SeedSequence([14121256, cfg, *extra])``.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 14121256


def rng_for(cfg: int, *extra: int) -> np.random.Generator:
    """Generator for workload ``cfg`` (1..5, or >=100 for test signals)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, int(cfg), *map(int, extra)])))


# ----------------------------------------------------------------------------------------------
# quantiser and packer
# ----------------------------------------------------------------------------------------------

def quantize(x: np.ndarray, bits: int, sigma: float = 1.0) -> np.ndarray:
    """Sampler quantiser: float samples -> uint8 codes (or float32 for bits=32)."""
    x = np.asarray(x, dtype=np.float64)
    if bits == 2:
        th = sigma
        return ((x >= -th).astype(np.uint8) + (x >= 0.0).astype(np.uint8) + (x >= th).astype(np.uint8))
    if bits == 4:
        step = 0.5 * sigma
        return np.clip(np.floor(x / step) + 8.0, 0, 15).astype(np.uint8)
    if bits == 8:
        return np.clip(np.rint(x), -128, 127).astype(np.int8).view(np.uint8)
    if bits == 32:
        return x.astype(np.float32)
    raise ValueError(f"unsupported bits={bits}")


def pack_codes(codes: np.ndarray, bits: int) -> np.ndarray:
    """Pack codes shaped [T, S] (time-major) into the wire byte layout."""
    codes = np.ascontiguousarray(codes)
    if bits == 32:
        return codes.astype("<f4").reshape(-1).view(np.uint8).copy()
    flat = codes.reshape(-1).astype(np.uint8)
    if bits == 8:
        return flat.copy()
    per = 8 // bits
    if flat.size % per:
        raise ValueError("item count is not a whole number of bytes")
    mask = (1 << bits) - 1
    g = (flat & mask).reshape(-1, per).astype(np.uint16)
    out = np.zeros(g.shape[0], dtype=np.uint16)
    for i in range(per):
        out |= g[:, i] << (i * bits)
    return out.astype(np.uint8)


def _instance(packed, bits, n_streams, fft_len, n_frames, window="rect", pairs=None, **extra):
    if pairs is None:
        pairs = [(0, 1)] if n_streams == 2 else [(0, 2), (1, 3)]
    d = dict(packed=packed, bits=bits, n_streams=n_streams, fft_len=fft_len, n_frames=n_frames,
             n_samples=fft_len * n_frames, window=window, pairs=pairs, sample_rate_hz=16e6)
    d.update(extra)
    return d


# ----------------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------------

def make_tiny(n_frames: int = 64, fft_len: int = 1024, rho: float = 0.3, tone_bin: int = 100,
              tone_amp: float = 0.1, bits: int = 2, seed_extra: int = 0):
    """Tiny plain case: two 2-bit streams, correlation rho, common tone at a channel, Hann window.

    x = sqrt(1-rho) a + sqrt(rho) c + tone, y = sqrt(1-rho) b + sqrt(rho) c + tone, a, b, c iid N(0,1);
    tone = tone_amp * sin(2 pi tone_bin n / fft_len); thresholds at +-1 sigma (sigma = 1).
    """
    rng = rng_for(1, seed_extra)
    T = n_frames * fft_len
    a, b, c = rng.standard_normal((3, T))
    n = np.arange(T, dtype=np.float64)
    tone = tone_amp * np.sin(2.0 * np.pi * tone_bin * (n % fft_len) / fft_len)
    x = math.sqrt(1 - rho) * a + math.sqrt(rho) * c + tone
    y = math.sqrt(1 - rho) * b + math.sqrt(rho) * c + tone
    ts = np.stack([x, y], axis=1)
    if bits == 8:
        ts = ts * 16.0
    codes = quantize(ts, bits, sigma=1.0)
    return _instance(pack_codes(codes, bits), bits, 2, fft_len, n_frames, window="hann")


def _line_model(n_bins: int, C: int, rho: float, line_peak: float = 0.01, line_fwhm: float = 20.0,
                v_scale: float = 1e-3):
    """Per-bin Stokes model: flat continuum + 3 Gaussian lines, V = v_scale * dI/dk, U = rho (continuum)."""
    k = np.arange(n_bins, dtype=np.float64)
    s = line_fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    I = np.ones(n_bins)
    dI = np.zeros(n_bins)
    for c0 in (C / 4, C / 2, 3 * C / 4):
        g = line_peak * np.exp(-0.5 * ((k - c0) / s) ** 2)
        I += g
        dI += -g * (k - c0) / s ** 2
    Q = np.zeros(n_bins)
    U = np.full(n_bins, rho)
    V = v_scale * dI
    return I, Q, U, V


def _colour_pair(rng, XX, YY, XY, n_bins):
    """Draw one frame's spectra (X_k, Y_k) with per-bin coherency [[XX, XY], [conj XY, YY]]."""
    l00 = np.sqrt(XX)
    l10 = np.conj(XY) / l00
    l11 = np.sqrt(np.maximum(YY - np.abs(XY) ** 2 / XX, 0.0))
    z = (rng.standard_normal((2, n_bins)) + 1j * rng.standard_normal((2, n_bins))) * math.sqrt(0.5)
    X = l00 * z[0]
    Y = l10 * z[0] + l11 * z[1]
    # DC and Nyquist bins of a real signal are real
    for idx in (0, n_bins - 1):
        X[idx] = math.sqrt(2.0) * X[idx].real
        Y[idx] = math.sqrt(2.0) * Y[idx].real
    return X, Y


def _spectral_streams(rng, fft_len, n_frames, XX, YY, XY, sigma, tone=None):
    """Time series [T, 2] whose per-frame spectra follow the coherency; optional extra tone (amp, bin, phase)."""
    n_bins = fft_len // 2 + 1
    out = np.empty((n_frames * fft_len, 2), dtype=np.float64)
    n = np.arange(fft_len, dtype=np.float64)
    tone_sig = None
    if tone is not None:
        amp, kt, ph = tone
        tone_sig = amp * sigma * np.cos(2.0 * np.pi * kt * n / fft_len + ph)
    for f in range(n_frames):
        X, Y = _colour_pair(rng, XX, YY, XY, n_bins)
        x = np.fft.irfft(X, n=fft_len, norm="ortho") * sigma
        y = np.fft.irfft(Y, n=fft_len, norm="ortho") * sigma
        if tone_sig is not None:
            x = x + tone_sig
            y = y + tone_sig
        out[f * fft_len:(f + 1) * fft_len, 0] = x
        out[f * fft_len:(f + 1) * fft_len, 1] = y
    return out


def make_paper(n_frames: int = 61, fft_len: int = 2 ** 18, rho: float = 0.05, sigma_lsb: float = 16.0,
               seed_extra: int = 0):
    """Paper-shaped case: two int8 streams at 16 Msps, 2^18-point frames, 61 frames (0.999424 s).

    Per frame and bin, spectra are drawn with coherency I+Q, I-Q, U+iV where I = 1 + three Gaussian lines
    (FWHM 20 ch, peak 0.01 of the continuum, at C/4, C/2, 3C/4), Q = 0, U = rho, V = 1e-3 dI/dk.
    """
    rng = rng_for(2, seed_extra)
    C = fft_len // 2
    n_bins = C + 1
    I, Q, U, V = _line_model(n_bins, C, rho)
    ts = _spectral_streams(rng, fft_len, n_frames, I + Q, I - Q, U + 1j * V, sigma_lsb)
    codes = quantize(ts, 8)
    return _instance(pack_codes(codes, 8), 8, 2, fft_len, n_frames, window="rect",
                     model=dict(I=I[:C], Q=Q[:C], U=U[:C], V=V[:C]))


def make_precision(n_frames: int = 610, fft_len: int = 2 ** 18, rho: float = 0.05, sigma_lsb: float = 16.0,
                   tone_db: float | None = None, tone_bin: float = 43690.0, seed_extra: int = 0):
    """Precision-form case: 4 int8 streams X0, X1, Y0, Y1 (pairs (0,2), (1,3)), 2^18 points.

    tone_db adds a tone of per-channel SNR tone_db to every stream: amplitude
    A = 2 * sigma * 10**(tone_db/20) / sqrt(N) (bin-centred when tone_bin is an integer).
    """
    rng = rng_for(3, seed_extra)
    C = fft_len // 2
    n_bins = C + 1
    I, Q, U, V = _line_model(n_bins, C, rho)
    tone = None
    if tone_db is not None:
        amp = 2.0 * 10 ** (tone_db / 20.0) / math.sqrt(fft_len)
        tone = (amp, tone_bin, 0.3)
    T = n_frames * fft_len
    codes = np.empty((T, 4), dtype=np.uint8)
    for band in range(2):
        ts = _spectral_streams(rng, fft_len, n_frames, I + Q, I - Q, U + 1j * V, sigma_lsb, tone=tone)
        q = quantize(ts, 8)
        codes[:, band] = q[:, 0]       # X_band
        codes[:, 2 + band] = q[:, 1]   # Y_band
    return _instance(pack_codes(codes, 8), 8, 4, fft_len, n_frames, window="rect", pairs=[(0, 2), (1, 3)])


MODES = {
    # Table 1: IF bandwidth, sampling rate, code width, FFT length (channels = N / 2), four IFs X0, X1, Y0, Y1
    "8MHz": dict(bits=4, fft_len=2 ** 18, sample_rate_hz=16e6),
    "4MHz": dict(bits=8, fft_len=2 ** 17, sample_rate_hz=8e6),
}


def make_mode(mode: str, n_frames: int = 61, rho: float = 0.05, seed_extra: int = 0):
    """One of the sampler modes of Table 1 with its four IFs X0, X1, Y0, Y1 (pairs (0, 2), (1, 3)): per
    band, the paper-shaped line model (see make_paper) quantised by that mode's sampler (4-bit: step sigma/2;
    8-bit: sigma = 16 LSB).  61 frames are 0.999 s of data in either mode."""
    m = MODES[mode]
    rng = rng_for(6, seed_extra, m["bits"])
    N = m["fft_len"]
    C = N // 2
    I, Q, U, V = _line_model(C + 1, C, rho)
    sigma = 16.0 if m["bits"] == 8 else 1.0
    T = n_frames * N
    codes = np.empty((T, 4), dtype=np.uint8)
    for band in range(2):
        ts = _spectral_streams(rng, N, n_frames, I + Q, I - Q, U + 1j * V, sigma)
        q = quantize(ts, m["bits"], sigma=sigma)
        codes[:, band] = q[:, 0]       # X_band
        codes[:, 2 + band] = q[:, 1]   # Y_band
    d = _instance(pack_codes(codes, m["bits"]), m["bits"], 4, N, n_frames, window="rect", pairs=[(0, 2), (1, 3)])
    d["sample_rate_hz"] = m["sample_rate_hz"]
    return d


def make_correlated_noise(bits: int, rho: float, fft_len: int, n_frames: int, cfg: int = 100,
                          seed_extra: int = 0, window: str = "rect"):
    """Two streams of N(0,1) noise with correlation rho, quantised (sigma = 1; 8-bit uses 16 LSB)."""
    rng = rng_for(cfg, seed_extra, bits)
    T = fft_len * n_frames
    a, b, c = rng.standard_normal((3, T))
    x = math.sqrt(1 - rho) * a + math.sqrt(rho) * c
    y = math.sqrt(1 - rho) * b + math.sqrt(rho) * c
    ts = np.stack([x, y], axis=1)
    if bits == 8:
        ts = ts * 16.0
    codes = quantize(ts, bits, sigma=1.0)
    return _instance(pack_codes(codes, bits), bits, 2, fft_len, n_frames, window=window)


def batching_params(n_inst: int = 64, e_range=(12, 20), f_range=(8, 256), seed_extra: int = 0):
    """Shapes of the batching-form set: log2 N uniform on e_range, frames uniform on f_range, 2- or 8-bit with
    probability 1/2, correlation rho ~ U(0, 0.5)."""
    rng = rng_for(4, seed_extra)
    e = rng.integers(e_range[0], e_range[1] + 1, size=n_inst)
    F = rng.integers(f_range[0], f_range[1] + 1, size=n_inst)
    bits = np.where(rng.random(n_inst) < 0.5, 2, 8)
    rho = rng.uniform(0.0, 0.5, size=n_inst)
    return e, F, bits, rho


def make_batching(n_inst: int = 64, e_range=(12, 20), f_range=(8, 256), max_frames: int | None = None,
                  seed_extra: int = 0):
    """Batching-form set: uneven instances, N = 2^e (e uniform), frames uniform, 2/8-bit mix, rho ~ U(0, .5)."""
    e, F, bits, rho = batching_params(n_inst, e_range, f_range, seed_extra)
    out = []
    for i in range(n_inst):
        Fi = int(F[i]) if max_frames is None else int(min(F[i], max_frames))
        d = make_correlated_noise(int(bits[i]), float(rho[i]), 1 << int(e[i]), Fi, cfg=4, seed_extra=1000 + i)
        d["rho"] = float(rho[i])
        out.append(d)
    return out


def make_tone_f32(fft_len: int, n_frames: int, k0: float, amp: float = 1.0, phase: float = 0.0,
                  phase_y: float | None = None, amp_y: float | None = None):
    """Float32 two-stream pure tone x = amp cos(2 pi k0 n / N + phase) (frame-periodic for integer k0)."""
    T = fft_len * n_frames
    n = np.arange(T, dtype=np.float64)
    x = amp * np.cos(2.0 * np.pi * k0 * n / fft_len + phase)
    ay = amp if amp_y is None else amp_y
    py = phase if phase_y is None else phase_y
    y = ay * np.cos(2.0 * np.pi * k0 * n / fft_len + py)
    codes = quantize(np.stack([x, y], axis=1), 32)
    return _instance(pack_codes(codes, 32), 32, 2, fft_len, n_frames)


def make_identical_streams(bits: int, fft_len: int, n_frames: int, seed_extra: int = 0):
    """Both streams carry the same quantised noise."""
    rng = rng_for(101, seed_extra, bits)
    x = rng.standard_normal(fft_len * n_frames)
    if bits == 8:
        x = x * 16.0
    codes = quantize(np.stack([x, x], axis=1), bits, sigma=1.0)
    return _instance(pack_codes(codes, bits), bits, 2, fft_len, n_frames)


def make_fully_polarized_f32(fft_len: int, n_frames: int, alpha: complex = 0.6 - 0.45j, seed_extra: int = 0):
    """Float32 pair with Y_k = alpha X_k in every frame (DC and Nyquist zero): a fully polarised signal."""
    rng = rng_for(102, seed_extra)
    n_bins = fft_len // 2 + 1
    T = fft_len * n_frames
    xs = np.empty((T, 2))
    for f in range(n_frames):
        X = rng.standard_normal(n_bins) + 1j * rng.standard_normal(n_bins)
        X[0] = 0.0
        X[-1] = 0.0
        Y = alpha * X
        xs[f * fft_len:(f + 1) * fft_len, 0] = np.fft.irfft(X, n=fft_len, norm="ortho")
        xs[f * fft_len:(f + 1) * fft_len, 1] = np.fft.irfft(Y, n=fft_len, norm="ortho")
    codes = quantize(xs, 32)
    return _instance(pack_codes(codes, 32), 32, 2, fft_len, n_frames, alpha=alpha)


def make_differentiation(n_frames: int = 128, fft_len: int = 2 ** 16, sigma_lsb: float = 16.0,
                         q_frac: float = 0.1, u_frac: float = 0.05, gain_sd: float = 0.05, d_amp: float = 0.02,
                         seed_extra: int = 0):
    """Differentiation-form case: a calibrator observed through true gains and leakage.

    Calibrator: flat I = 1, Q = q_frac, U = u_frac, V = 0 (linear feeds, parallactic angle 0).  Observed
    voltages are v' = G J v with G = diag(g_x[k], g_y[k]), g = 1 + N(0, gain_sd^2) complex per channel, and
    J = [[1, d_x], [d_y, 1]] with |d| = d_amp and random phases, so the observed coherency is G J C J^H G^H.
    Also returns an independent initial guess for the gains, and the target Stokes spectra.
    """
    rng = rng_for(5, seed_extra)
    C = fft_len // 2
    n_bins = C + 1
    I, Q, U, V = 1.0, q_frac, u_frac, 0.0
    Cm = np.array([[I + Q, U + 1j * V], [U - 1j * V, I - Q]], dtype=np.complex128)

    def cgauss(shape, sd):
        return sd * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)

    gx = 1.0 + cgauss(n_bins, gain_sd)
    gy = 1.0 + cgauss(n_bins, gain_sd)
    ph = rng.uniform(0, 2 * np.pi, size=2)
    dx = d_amp * np.exp(1j * ph[0])
    dy = d_amp * np.exp(1j * ph[1])
    J = np.array([[1.0, dx], [dy, 1.0]], dtype=np.complex128)
    E = np.zeros((n_bins, 2, 2), dtype=np.complex128)
    E[:, 0, 0] = gx
    E[:, 0, 1] = gx * dx
    E[:, 1, 0] = gy * dy
    E[:, 1, 1] = gy
    M = E @ Cm @ np.conj(np.transpose(E, (0, 2, 1)))
    ts = _spectral_streams(rng, fft_len, n_frames, M[:, 0, 0].real, M[:, 1, 1].real, M[:, 0, 1], sigma_lsb)
    codes = quantize(ts, 8)
    gx0 = 1.0 + cgauss(C, gain_sd)
    gy0 = 1.0 + cgauss(C, gain_sd)
    target = np.zeros((1, 4, C))
    # the calibrator's Stokes in units of the observed power (sigma_lsb^2 per unit coherency)
    target[0, 0] = I * sigma_lsb ** 2
    target[0, 1] = Q * sigma_lsb ** 2
    target[0, 2] = U * sigma_lsb ** 2
    target[0, 3] = V * sigma_lsb ** 2
    return _instance(pack_codes(codes, 8), 8, 2, fft_len, n_frames, window="taps",
                     true_gain_x=gx[:C], true_gain_y=gy[:C], true_dterms=np.array([dx, dy]),
                     init_gain_x=gx0, init_gain_y=gy0, target=target)
