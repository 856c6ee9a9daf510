"""Oracle pins for the post-integration reductions: channel averaging with flagging (Sec. 4), the smoothed
bandpass and the bandpass variation (Sec. 3.3.2), band statistics and the Allan variances of Eq. 3 / Eq. 4
(Sec. 3.3.1, 3.3.3)."""
import os

import numpy as np
import pytest
from scipy import interpolate

from oracle import post

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def paper_value(name):
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith(name + " "):
                return float(line.split()[1])
    raise KeyError(name)


# ---------------------------------------------------------------------------------------- averaging
def test_average_factors_give_the_papers_resolutions():
    # 131072 channels over 8 MHz -> 32-channel bins; 16384 over 4 MHz -> 16-channel bins
    assert abs(32 * 8e6 / 131072 / 1e3 - paper_value("avg_resolution_khz_tmc1")) < 0.01
    assert abs(16 * 4e6 / 16384 / 1e3 - paper_value("avg_resolution_khz_rleo")) < 0.01
    assert 256 * 8e6 / 131072 / 1e3 == paper_value("bp_variation_average_khz")
    assert paper_value("bp_variation_average_channels") == 256


def test_constant_and_ramp_closed_forms():
    C, M = 4096, 32
    out, cnt = post.channel_average(np.full((2, C), 3.25), M)
    assert np.all(out == 3.25) and np.all(cnt == M)
    a, b = 0.37, -2.0
    ramp = a * np.arange(C) + b
    out, _ = post.channel_average(ramp, M)
    centres = np.arange(C // M) * M + (M - 1) / 2
    assert np.allclose(out[0], a * centres + b, rtol=0, atol=1e-12)
    # no flags: the bins carry the whole sum
    x = np.random.default_rng(1).standard_normal((3, C))
    out, _ = post.channel_average(x, M)
    assert np.allclose(out.sum(axis=1) * M, x.sum(axis=1), atol=1e-10)


def test_flagged_spike_is_excluded():
    C, M, k = 1024, 32, 517
    x = np.ones((1, C))
    x[0, k] = 1e9
    flags = np.zeros(C, dtype=np.uint8)
    flags[k] = 1
    out, cnt = post.channel_average(x, M, flags)
    assert np.all(out == 1.0)
    assert cnt[0, k // M] == M - 1 and np.sum(cnt) == C - 1
    out2, _ = post.channel_average(x, M)
    assert abs(out2[0, k // M] - (1 + (1e9 - 1) / M)) < 1e-6


def test_all_flagged_bin_and_non_finite_channels():
    x = np.arange(64, dtype=np.float64)[None].repeat(2, axis=0)
    x[1, 3] = np.nan
    flags = np.zeros(64, dtype=np.uint8)
    flags[8:16] = 1
    out, cnt = post.channel_average(x, 8, flags)
    assert np.isnan(out[0, 1]) and cnt[0, 1] == 0
    assert cnt[1, 0] == 7 and out[1, 0] == (np.sum(np.arange(8)) - 3) / 7


# ---------------------------------------------------------------------------------------- bandpass
def test_fit_range_matches_the_papers_edges():
    c0, c1 = post.fit_range(131072, paper_value("bp_edge_fraction"))
    assert (c0, c1) == (7864, 131072 - 7864)


def test_spline_reproduces_cubics_exactly():
    C = 8192
    c = np.arange(C, dtype=np.float64)
    u = c / C
    h = 2.0 + 0.5 * u - 1.3 * u ** 2 + 0.7 * u ** 3
    sm, _ = post.bandpass_fit(h, 128, 0.06)
    c0, c1 = post.fit_range(C, 0.06)
    assert np.all(np.isnan(sm[:c0])) and np.all(np.isnan(sm[c1:]))
    assert np.max(np.abs(sm[c0:c1] - h[c0:c1])) < 1e-12


@pytest.mark.parametrize("C,K", [(8192, 128), (131072, 128), (5000, 96)])
def test_spline_equals_library_least_squares_spline(C, K):
    rng = np.random.default_rng(C)
    c = np.arange(C, dtype=np.float64)
    h = 1 + 0.1 * np.sin(c / 700.0) + 0.01 * rng.standard_normal(C)
    sm, coef = post.bandpass_fit(h, K, 0.06)
    c0, c1 = post.fit_range(C, 0.06)
    n_int = -(-(c1 - c0) // K)
    t = c0 + K * np.arange(-3, n_int + 4, dtype=np.float64)
    spl = interpolate.make_lsq_spline(c[c0:c1], h[c0:c1], t, k=3)
    assert np.max(np.abs(spl.c - coef)) < 1e-9
    assert np.max(np.abs(spl(c[c0:c1]) - sm[c0:c1])) < 1e-10


def test_spline_noise_reduction_matches_projection_theory():
    """Least squares onto nb basis functions keeps nb of the n_pts noise degrees of freedom:
    E mean (fit - truth)^2 = sigma^2 nb / n_pts."""
    C, K, sigma = 131072, 128, 0.01
    rng = np.random.default_rng(5)
    c = np.arange(C, dtype=np.float64)
    truth = 1 + 0.2 * np.cos(c / 9000.0)
    sm, coef = post.bandpass_fit(truth + sigma * rng.standard_normal(C), K, 0.06)
    c0, c1 = post.fit_range(C, 0.06)
    got = np.mean((sm[c0:c1] - truth[c0:c1]) ** 2)
    expect = sigma ** 2 * coef.size / (c1 - c0)
    assert abs(got / expect - 1) < 0.1


def test_bandpass_correct_of_scaled_bandpass_is_one():
    rng = np.random.default_rng(2)
    H = 1 + rng.random(1000)
    G = np.array([0.5, 2.0, 1.25])
    hat = post.bandpass_correct(G[:, None] * H[None], H, G)
    assert np.max(np.abs(hat - 1)) < 1e-15


def test_band_stats_equal_library_moments():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 3000)) * 0.1 + 1
    x[2, 100:200] = np.nan
    st = post.band_stats(x)
    for s in range(4):
        v = x[s][np.isfinite(x[s])]
        assert abs(st[s, 0] - np.mean(v)) < 1e-14 and abs(st[s, 1] - np.std(v)) < 1e-14


# ---------------------------------------------------------------------------------------- Allan variances
def test_allan_of_linear_drift_is_zero_and_of_quadratic_is_closed_form():
    t = np.arange(2000, dtype=np.float64)
    lags = [1, 2, 7, 64, 500]
    lin = post.allan(3.0 + 0.01 * t, lags, spacing=1.0)
    assert np.max(np.abs(lin)) < 1e-20
    q = 1e-4
    quad = post.allan(q * t ** 2, lags, spacing=0.5)
    # second difference 2 q L^2 at every t: sigma^2 = (2 q L^2)^2 / (2 (L spacing)^2)
    expect = np.array([(2 * q * L * L) ** 2 / (2 * (L * 0.5) ** 2) for L in lags])
    assert np.max(np.abs(quad[0] / expect - 1)) < 1e-9


def test_allan_of_white_noise_is_three_sigma_squared_over_lag_squared():
    """White noise of variance s^2: E(x[t+L] - 2x[t] + x[t-L])^2 = 6 s^2, so sigma^2 = 3 s^2 / tau^2 (Sec.
    3.3.3 gives 3 sigma^2 / dnu^2 for a white-noise spectrum)."""
    s, n = 0.02, 400000
    x = 1 + s * np.random.default_rng(7).standard_normal(n)
    lags = [1, 3, 16]
    got = post.allan(x, lags, spacing=2.0)[0]
    expect = np.array([3 * s * s / (L * 2.0) ** 2 for L in lags])
    assert np.max(np.abs(got / expect - 1)) < 0.02
    gn = post.allan(5 * x, lags, spacing=2.0, normalize=True)[0]
    assert np.max(np.abs(gn / got - 1)) < 0.01  # normalised by the mean (about 1 here)


def test_allan_skips_triples_with_non_finite_samples():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(50)
    x[20] = np.nan
    for L in (1, 4):
        terms = [(x[t + L] - 2 * x[t] + x[t - L]) ** 2 for t in range(L, 50 - L)
                 if np.isfinite(x[t + L]) and np.isfinite(x[t]) and np.isfinite(x[t - L])]
        got = post.allan(x, [L])[0, 0]
        assert abs(got - sum(terms) / len(terms) / (2.0 * L * L)) < 1e-12
    assert np.isnan(post.allan(x, [25])[0, 0])  # no t with t - L >= 0 and t + L < 50
