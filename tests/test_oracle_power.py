"""Pins of the oracle's level histograms and total-power estimates (Sec. 2: total power from the samplers'
bit distributions): hand-counted bytes, sample totals, and the closed forms of a quantised Gaussian."""
import math

import numpy as np
import pytest

import oracle
import synth


def test_hand_counted_2bit():
    # codes of (x, y) per time step, LSB first: byte 0b11_10_01_00 holds t0 = (0, 1), t1 = (2, 3)
    packed = np.array([0b11100100, 0b00000000, 0b11111111], dtype=np.uint8)
    c = oracle.level_histograms(packed, 2, 2, 6, [(0, 1)])
    # x codes: 0, 2, 0, 0, 3, 3; y codes: 1, 3, 0, 0, 3, 3
    assert c[0, 0].tolist() == [3, 0, 1, 2]
    assert c[0, 1].tolist() == [2, 1, 0, 3]


def test_hand_counted_int8_two_pairs():
    t = np.array([[-128, 5, 127, -1], [5, 5, -1, 0]], dtype=np.int8)  # two time steps, four streams
    c = oracle.level_histograms(t.reshape(-1).view(np.uint8), 8, 4, 2, [(0, 2), (1, 3)])
    assert c.sum(axis=2).tolist() == [[2, 2], [2, 2]]
    assert c[0, 0, 0] == 1 and c[0, 0, 128 + 5] == 1          # stream 0: -128, 5
    assert c[0, 1, 255] == 1 and c[0, 1, 127] == 1            # stream 2: 127, -1
    assert c[1, 0, 133] == 2                                   # stream 1: 5, 5
    assert c[1, 1, 127] == 1 and c[1, 1, 128] == 1            # stream 3: -1, 0


@pytest.mark.parametrize("bits", [2, 4, 8])
def test_counts_sum_to_samples(bits):
    d = synth.make_correlated_noise(bits, 0.3, 256, 16, seed_extra=bits)
    c = oracle.level_histograms(d["packed"], bits, 2, d["n_samples"], d["pairs"])
    assert c.sum(axis=2).tolist() == [[d["n_samples"], d["n_samples"]]]


def test_two_bit_sigma_over_threshold_closed_form():
    # Gaussian of sigma = theta / k quantised at +-theta: P(|x| < theta) = erf(k / sqrt 2), so the estimate
    # returns 1 / k within the binomial error of P
    rng = np.random.default_rng(11)
    n = 1 << 20
    for k in (0.5, 1.0, 1.7):
        x = rng.standard_normal((n, 2)) / k  # theta = 1
        codes = synth.quantize(x, 2, sigma=1.0)
        c = oracle.level_histograms(synth.pack_codes(codes, 2), 2, 2, n, [(0, 1)])
        est = oracle.total_power(c, 2)[0, :, 1]
        pin = math.erf(k / math.sqrt(2.0))
        # d(1/k)/dP ~ 1 / (k^2 sqrt(2 pi) exp(-k^2/2) / sqrt 2 ...): bound via the binomial sigma of P
        dp = 5 * math.sqrt(pin * (1 - pin) / n)
        lo = 1.0 / (math.sqrt(2) * float(__import__("scipy").special.erfinv(min(pin + dp, 0.999999))))
        hi = 1.0 / (math.sqrt(2) * float(__import__("scipy").special.erfinv(max(pin - dp, 1e-9))))
        assert np.all((est > lo) & (est < hi)), (k, est, lo, hi)


def test_int8_mean_square_level():
    # sigma = 16 LSB, rounding to integers: E[level^2] = sigma^2 + 1/12 (Sheppard), clipping negligible
    rng = np.random.default_rng(12)
    n = 1 << 20
    x = rng.standard_normal((n, 2)) * 16.0
    codes = synth.quantize(x, 8)
    c = oracle.level_histograms(synth.pack_codes(codes, 8), 8, 2, n, [(0, 1)])
    m2 = oracle.total_power(c, 8)[0, :, 0]
    assert np.all(np.abs(m2 - (256.0 + 1.0 / 12.0)) < 5 * 256.0 * math.sqrt(2.0 / n))
    assert np.all(np.isnan(oracle.total_power(c, 8)[0, :, 1]))
