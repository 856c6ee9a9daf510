"""Oracle pins for the segment transform (Sec. 2: FFT of each segment; Sec. 3.1: rectangular window)."""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def paper_value(name):
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith(name + " "):
                return float(line.split()[1])
    raise KeyError(name)


def _relnorm(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [2, 4, 8, 16, 64, 256, 1024])
def test_radix2_matches_brute_force_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert _relnorm(oracle.fft(x), oracle.dft(x)) < 1e-12


@pytest.mark.parametrize("n", [2 ** 10, 2 ** 14, 2 ** 18])
def test_radix2_matches_library_fft(n):
    rng = np.random.default_rng(n + 1)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert _relnorm(oracle.fft(x), np.fft.fft(x)) < 1e-12


@pytest.mark.parametrize("n", [16, 1024, 2 ** 16])
def test_parseval_real_input(n):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(n)
    X = oracle.fft(x)
    lhs = np.sum(x * x)
    rhs = (abs(X[0]) ** 2 + abs(X[n // 2]) ** 2 + 2 * np.sum(np.abs(X[1:n // 2]) ** 2)) / n
    assert abs(lhs - rhs) / lhs < 1e-12


@pytest.mark.parametrize("n,k0", [(1024, 100), (4096, 1), (2 ** 18, 43690)])
def test_pure_tone_rect(n, k0):
    A, phi = 0.75, 0.4
    t = np.arange(n)
    X = oracle.fft(A * np.cos(2 * np.pi * k0 * t / n + phi))
    expect = np.zeros(n // 2, dtype=complex)
    expect[k0] = A * n / 2 * np.exp(1j * phi)
    assert np.max(np.abs(X[: n // 2] - expect)) < 1e-9 * A * n


@pytest.mark.parametrize("n,k0", [(1024, 100), (8192, 2000)])
def test_pure_tone_periodic_hann(n, k0):
    A, phi = 1.3, -1.1
    w, s2 = oracle.window("hann", n)
    assert abs(s2 / n - 0.375) < 1e-12  # periodic Hann: mean of w^2 is 3/8
    t = np.arange(n)
    X = oracle.fft(w * A * np.cos(2 * np.pi * k0 * t / n + phi))
    expect = np.zeros(n // 2, dtype=complex)
    expect[k0] = A * n / 4 * np.exp(1j * phi)
    expect[k0 - 1] = -A * n / 8 * np.exp(1j * phi)
    expect[k0 + 1] = -A * n / 8 * np.exp(1j * phi)
    assert np.max(np.abs(X[: n // 2] - expect)) < 1e-9 * A * n


def test_off_bin_complex_tone_is_dirichlet_kernel():
    n, k0 = 512, 37.3
    t = np.arange(n)
    X = oracle.fft(np.exp(2j * np.pi * k0 * t / n))
    d = np.arange(n) - k0
    expect = np.abs(np.sin(np.pi * d) / np.sin(np.pi * d / n))
    assert np.max(np.abs(np.abs(X) - expect)) < 1e-9 * n


def test_tone_sweep_fwhm_matches_paper():
    """Sec. 3.1: sweeping a tone across a channel traces sinc^2 with FWHM 0.886 channel (54.07 Hz)."""
    n, ref = 4096, 1000
    t = np.arange(n)
    offs = np.linspace(-1.0, 1.0, 401)
    resp = []
    for d in offs:
        X = oracle.fft(np.cos(2 * np.pi * (ref + d) * t / n))
        resp.append(abs(X[ref]) ** 2)
    resp = np.array(resp) / max(resp)
    # half-power crossings by linear interpolation on each side
    half = 0.5
    i_r = np.where((offs > 0) & (resp < half))[0][0]
    i_l = np.where((offs < 0) & (resp >= half))[0][0]
    xr = offs[i_r - 1] + (half - resp[i_r - 1]) * (offs[i_r] - offs[i_r - 1]) / (resp[i_r] - resp[i_r - 1])
    xl = offs[i_l - 1] + (half - resp[i_l - 1]) * (offs[i_l] - offs[i_l - 1]) / (resp[i_l] - resp[i_l - 1])
    fwhm = xr - xl
    assert abs(fwhm - paper_value("sinc2_fwhm_channels")) < 1e-3
    spacing = 16e6 / 2 ** 18
    assert abs(fwhm * spacing - paper_value("sinc2_fwhm_hz_8mhz")) < 0.05
    assert round(spacing) == paper_value("channel_spacing_hz")


def test_taps_window_interpolates_control_points():
    n = 1024
    taps = np.linspace(0.5, 1.5, 64) ** 2
    w, s2 = oracle.window("taps", n, taps=taps)
    assert w[0] == taps[0] and w[-1] == taps[-1]
    # a linear ramp of taps gives a linear window
    w2, _ = oracle.window("taps", n, taps=np.linspace(0.0, 63.0, 64))
    assert np.max(np.abs(w2 - np.arange(n) * 63.0 / (n - 1))) < 1e-12
    # all-ones taps is the rectangular window
    w3, s3 = oracle.window("taps", n, taps=np.ones(64))
    assert np.all(w3 == 1.0) and s3 == n
    assert abs(s2 - np.sum(w * w)) < 1e-9
