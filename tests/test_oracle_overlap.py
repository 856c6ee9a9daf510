"""Oracle pins for overlapped segmentation and the offline apodisation windows (Sec. 3.1: frames with 50 %
overlap; Hanning, Hamming and Blackman windows applied offline).

Windows are the periodic (DFT-even) forms.  Pins: the library's periodic windows, the closed-form sums of
squares, and the exact three- or five-channel response of a channel-centred cosine.  Segmentation: frame f
covers samples f*hop .. f*hop + N - 1, so an overlapped integration is the sum of contiguous integrations
of shifted copies of the stream, and the frame count is (T - N) / hop + 1.
"""
import numpy as np
import pytest
from scipy import signal

import oracle
import synth

COEF = {"hann": (0.5, 0.5), "hamming": (0.54, 0.46), "blackman": (0.42, 0.5, 0.08)}


@pytest.mark.parametrize("kind", ["hann", "hamming", "blackman"])
def test_windows_match_library_periodic_windows(kind):
    for n in (256, 1024, 4096):
        w, s2 = oracle.window(kind, n)
        ref = signal.get_window(kind, n, fftbins=True)
        assert np.max(np.abs(w - ref)) < 1e-15
        # sum of squares of a cosine-sum window over whole periods: a0^2 + sum_j a_j^2 / 2 per sample
        a = COEF[kind]
        assert abs(s2 - n * (a[0] ** 2 + sum(x * x for x in a[1:]) / 2)) < 1e-9 * n


def _cosine_f32(n_time, N, k0, amp, n_streams=2):
    t = np.arange(n_time)
    x = (amp * np.cos(2 * np.pi * k0 * t / N)).astype(np.float32)
    return np.repeat(x[:, None], n_streams, axis=1).reshape(-1).view(np.uint8), x


@pytest.mark.parametrize("kind", ["hann", "hamming", "blackman"])
def test_channel_centred_cosine_response(kind):
    """A cosine at channel k0 (whole periods per frame) under a cosine-sum window with coefficients
    a0, a1, a2 has X[k0] = A N/2 a0, X[k0 +- j] = (-1)^j A N/2 a_j / 2 and nothing else."""
    N, F, k0, A = 1024, 3, 200, 3.0
    packed, _ = _cosine_f32(N * F, N, k0, A)
    w, s2 = oracle.window(kind, N)
    acc, nf = oracle.accumulate(packed, 32, 2, N * F, N, w, [(0, 1)])
    assert nf == F
    a = COEF[kind]
    amp = np.zeros(N // 2)
    amp[k0] = A * N / 2 * a[0]
    for j in range(1, len(a)):
        amp[k0 - j] = amp[k0 + j] = (-1) ** j * A * N / 2 * a[j] / 2
    expect = F * amp ** 2
    peak = expect[k0]
    for q in (0, 1, 2):  # XX*, YY*, Re XY*: identical streams
        assert np.max(np.abs(acc[0, q] - expect)) < 1e-6 * peak, q
    assert np.max(np.abs(acc[0, 3])) < 1e-6 * peak


@pytest.mark.parametrize("j", [1, 2, 3])
def test_overlapped_is_sum_of_shifted_contiguous_integrations(j):
    N, F = 512, 6
    hop = N >> j
    inst = synth.make_correlated_noise(8, 0.3, N, F, seed_extra=70 + j)
    w, _ = oracle.window("hann", N)
    T = inst["n_samples"]
    acc, nf = oracle.accumulate(inst["packed"], 8, 2, T, N, w, [(0, 1)], hop=hop)
    assert nf == (T - N) // hop + 1 == (1 << j) * F - ((1 << j) - 1)
    total = np.zeros_like(acc)
    frames = 0
    bytes_per_sample = 2  # two int8 streams
    for q in range(1 << j):
        start = q * hop
        n = (T - start) // N * N
        part, f = oracle.accumulate(inst["packed"][start * bytes_per_sample:(start + n) * bytes_per_sample], 8, 2,
                                    n, N, w, [(0, 1)])
        total += part
        frames += f
    assert frames == nf
    assert np.max(np.abs(acc - total)) <= 1e-12 * np.max(np.abs(total))


def test_hop_equal_to_fft_len_is_contiguous():
    inst = synth.make_correlated_noise(4, 0.2, 256, 5, seed_extra=3)
    w, _ = oracle.window("blackman", 256)
    a0, f0 = oracle.accumulate(inst["packed"], 4, 2, inst["n_samples"], 256, w, [(0, 1)])
    a1, f1 = oracle.accumulate(inst["packed"], 4, 2, inst["n_samples"], 256, w, [(0, 1)], hop=256)
    assert f0 == f1 == 5 and np.array_equal(a0, a1)


@pytest.mark.parametrize("hop", [3, 96, 512, -128])
def test_bad_hop_is_rejected(hop):
    inst = synth.make_correlated_noise(8, 0.2, 256, 4, seed_extra=4)
    w, _ = oracle.window("rect", 256)
    with pytest.raises(ValueError):
        oracle.accumulate(inst["packed"], 8, 2, inst["n_samples"], 256, w, [(0, 1)], hop=hop)
