"""Post-integration reductions on the GPU against the FP64 oracle (oracle/post.py), through the C ABI: channel
averaging with flags (Sec. 4), the smoothed bandpass and bandpass variation (Sec. 3.3.2), band moments and the
Allan variances of Eq. 3 and Eq. 4 (Sec. 3.3.1, 3.3.3).

Inputs are FP32 spectra (the library's Stokes output format); both sides compute in FP64.  Bounds: counts
bit-exact; FP32 outputs within 1e-6 relative of the oracle (one rounding to FP32 plus FP64 summation-order
differences); FP64 outputs (moments, Allan variances) within 1e-10 relative.
"""
import sys

import warnings

import numpy as np
import pytest

from oracle import post

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1412_1256_amd as pk
    pk.lib()
    return torch, pk, torch.device("cuda:0")


def rel_close(got, ref, rtol):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    m = ~np.isnan(ref)
    err = np.max(np.abs(got[m] - ref[m]) / np.maximum(np.abs(ref[m]), 1e-30)) if m.any() else 0.0
    assert err <= rtol, err
    return err


def spectra(n_spec, C, seed, nan_edges=0):
    rng = np.random.default_rng(seed)
    k = np.arange(C)
    x = (1 + 0.2 * np.sin(k / 5000.0))[None] * (1 + 0.01 * rng.standard_normal((n_spec, C)))
    x = x.astype(np.float32)
    if nan_edges:
        x[:, :nan_edges] = np.nan
        x[:, C - nan_edges:] = np.nan
    return x


@pytest.mark.parametrize("factor", [1, 16, 32, 96, 256, 4096, 8192])
def test_channel_average_with_flags(env, factor):
    torch, pk, dev = env
    C = 131072 if factor != 96 else 96 * 1000
    say(f"channel average factor={factor} C={C}")
    x = spectra(8, C, factor, nan_edges=100)
    flags = np.zeros(C, dtype=np.uint8)
    flags[[5, 777, C // 2, C // 2 + 1, C - 300]] = 1
    x[:, C // 2] = 1e9  # a spurious channel (flagged)
    out, cnt = pk.channel_average(torch.from_numpy(x).to(dev), factor, torch.from_numpy(flags).to(dev))
    torch.cuda.synchronize(dev)
    ref, rcnt = post.channel_average(x, factor, flags)
    assert np.array_equal(cnt.cpu().numpy(), rcnt)
    e = rel_close(out.cpu().numpy(), ref, 1e-6)
    say(f"  err {e}")


def test_channel_average_of_stokes_output(env):
    """The paper's TMC-1 reduction on the library's own Stokes output: 131072 channels to 4096 (1.95 kHz)."""
    torch, pk, dev = env
    import synth
    inst = synth.make_paper(n_frames=8)
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    plan.reset()
    plan.accumulate(torch.from_numpy(inst["packed"]).to(dev))
    st = plan.stokes()
    flags = torch.zeros(st.shape[-1], dtype=torch.uint8, device=dev)
    flags[65536] = 1
    out, cnt = pk.channel_average(st, 32, flags)
    torch.cuda.synchronize(dev)
    assert out.shape == (1, 4, 4096)
    ref, rcnt = post.channel_average(st.cpu().numpy().reshape(4, -1), 32, flags.cpu().numpy())
    assert np.array_equal(cnt.cpu().numpy().reshape(4, -1), rcnt)
    rel_close(out.cpu().numpy().reshape(4, -1), ref, 1e-6)


@pytest.mark.parametrize("C,K,edge", [(131072, 128, 0.06), (8192, 128, 0.06), (5000, 96, 0.1), (1 << 20, 512, 0.06),
                                      (4096, 64, 0.0)])
def test_bandpass_fit(env, C, K, edge):
    torch, pk, dev = env
    say(f"bandpass fit C={C} K={K} edge={edge}")
    rng = np.random.default_rng(C + K)
    k = np.arange(C)
    h = (1 + 0.3 * np.sin(k / (C / 7.0)) + 0.05 * np.cos(k / 311.0) + 0.01 * rng.standard_normal(C)).astype(np.float32)
    got = pk.bandpass_fit(torch.from_numpy(h).to(dev), K, edge).cpu().numpy()
    ref, _ = post.bandpass_fit(h, K, edge)
    e = rel_close(got, ref, 1e-6)
    say(f"  err {e}")


def test_bandpass_correct_and_stats(env):
    torch, pk, dev = env
    C = 131072
    hk = spectra(30, C, 3)
    smooth = post.bandpass_fit(hk.mean(axis=0), 128, 0.06)[0].astype(np.float32)
    G = 1 + 0.01 * np.arange(30)
    got = pk.bandpass_correct(torch.from_numpy(hk).to(dev), torch.from_numpy(smooth).to(dev),
                              torch.from_numpy(G).to(dev))
    st = pk.band_stats(got)
    torch.cuda.synchronize(dev)
    ref = post.bandpass_correct(hk, smooth, G)
    rel_close(got.cpu().numpy(), ref, 1e-6)
    # moments of the GPU's own FP32 output
    rel_close(st.cpu().numpy(), post.band_stats(got.cpu().numpy()), 1e-10)


def test_bandpass_stability_chain(env):
    """Sec. 3.3.2 end to end: a series of integrations H_k with gain drift, the long-integration bandpass
    smoothed (128-channel knots, 6 % edges), H^_k = H_k / (G_k H), 256-channel averages, their mean and SD."""
    torch, pk, dev = env
    C, K = 131072, 30
    rng = np.random.default_rng(11)
    k = np.arange(C)
    shape = 1 + 0.4 * np.exp(-((k - C / 2) / (C / 3)) ** 2) + 0.02 * np.sin(k / 900.0)
    G = 1 + 0.002 * np.arange(K)
    hk = (G[:, None] * shape[None] * (1 + 2.6e-3 * rng.standard_normal((K, C)))).astype(np.float32)
    # GPU chain
    t_hk = torch.from_numpy(hk).to(dev)
    H = t_hk.double().mean(dim=0).float()
    smooth = pk.bandpass_fit(H, 128, 0.06)
    hat = pk.bandpass_correct(t_hk, smooth, torch.from_numpy(G).to(dev))
    binned, cnt = pk.channel_average(hat, 256)
    st = pk.band_stats(binned).cpu().numpy()
    torch.cuda.synchronize(dev)
    # oracle chain from the same FP32 series (its own FP64 arithmetic at every stage)
    sm_ref, _ = post.bandpass_fit(H.cpu().numpy(), 128, 0.06)
    hat_ref = post.bandpass_correct(hk, sm_ref, G)
    bin_ref, _ = post.channel_average(hat_ref, 256)
    st_ref = post.band_stats(bin_ref)
    say(f"  mean, SD of the first spectra {st[:3].tolist()}")
    assert np.max(np.abs(st[:, 0] - st_ref[:, 0])) < 1e-6
    assert np.max(np.abs(st[:, 1] / st_ref[:, 1] - 1)) < 1e-3
    # white noise of 2.6e-3 per channel, 256-channel bins: SD about 2.6e-3 / 16
    assert np.all(np.abs(st[:, 1] / (2.6e-3 / 16) - 1) < 0.3)


def test_time_allan_variance_across_channels(env):
    """TAV (Eq. 3) of every channel of a series of 1-s integrations, normalised by the mean."""
    torch, pk, dev = env
    T, C = 1200, 4096
    rng = np.random.default_rng(4)
    x = (1 + 0.001 * np.arange(T)[:, None] / T + 0.01 * rng.standard_normal((T, C))).astype(np.float32)
    lags = [1, 2, 4, 8, 16, 64, 256, 599, 600]
    got = pk.allan(torch.from_numpy(x).to(dev), lags, spacing=1.0, normalize=True, axis=0).cpu().numpy()
    ref = post.allan(x.T, lags, spacing=1.0, normalize=True)
    rel_close(got, ref, 1e-10)
    assert np.all(np.isnan(got[:, -1]))  # 2 L >= n_points


def test_time_allan_variance_window_form(env):
    """TAV of side-by-side series with every lag at most 512 (the LDS-window form): the benchmark's lag set over
    1800 1-s integrations, normalised, and a lag set of two groups with a non-multiple-of-32 channel count."""
    torch, pk, dev = env
    rng = np.random.default_rng(11)
    T, C = 1800, 2048
    x = (1 + 0.002 * np.sin(np.arange(T) / 97.0)[:, None] + 0.01 * rng.standard_normal((T, C))).astype(np.float32)
    lags = [1, 2, 4, 8, 16, 64, 256, 512]
    got = pk.allan(torch.from_numpy(x).to(dev), lags, spacing=1.0, normalize=True, axis=0).cpu().numpy()
    rel_close(got, post.allan(x.T, lags, spacing=1.0, normalize=True), 1e-10)
    # a partial last workgroup (998 series, the window form) and an odd series count (999, the column form),
    # infinite samples (left out), lags in two groups of eight, and lags with one or no term
    for C in (998, 999):
        T = 777
        x = (3 + 0.05 * rng.standard_normal((T, C))).astype(np.float32)
        x[rng.integers(0, T, 200), rng.integers(0, C, 200)] = np.inf
        lags = [1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 377, 388, 389]
        got = pk.allan(torch.from_numpy(x).to(dev), lags, spacing=0.5, axis=0).cpu().numpy()
        ref = post.allan(x.T, lags, spacing=0.5)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        rel_close(got[ok], ref[ok], 1e-10)


def test_time_allan_variance_ragged_with_flags(env):
    """TAV of side-by-side series: a channel count that is not a whole number of 64-series workgroups, a
    series length that does not split evenly over the time slices, NaN (flagged) samples, both with and
    without normalisation; run twice, bitwise equal."""
    torch, pk, dev = env
    T, C = 1001, 1000
    rng = np.random.default_rng(9)
    x = (2 + 0.02 * rng.standard_normal((T, C))).astype(np.float32)
    x[rng.integers(0, T, 300), rng.integers(0, C, 300)] = np.nan
    x[:, 7] = np.nan  # a channel with no finite sample
    lags = [1, 3, 5, 17, 100, 250, 333, 499, 500, 501]
    xd = torch.from_numpy(x).to(dev)
    for normalize in (False, True):
        got = pk.allan(xd, lags, spacing=2.0, normalize=normalize, axis=0).cpu().numpy()
        again = pk.allan(xd, lags, spacing=2.0, normalize=normalize, axis=0).cpu().numpy()
        with warnings.catch_warnings():  # the mean of the all-NaN channel is NaN by design
            warnings.simplefilter("ignore", RuntimeWarning)
            ref = post.allan(x.T, lags, spacing=2.0, normalize=normalize)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        rel_close(got[ok], ref[ok], 1e-10)
        assert np.array_equal(np.nan_to_num(got), np.nan_to_num(again))
        assert np.all(np.isnan(got[7])) and np.all(np.isnan(got[:, -1]))


def test_spectral_allan_variance(env):
    """SAV (Eq. 4) along the channels of bandpass-corrected spectra with NaN band edges."""
    torch, pk, dev = env
    x = spectra(6, 131072, 8, nan_edges=7864)
    lags = [1, 2, 4, 16, 128, 1024]
    got = pk.allan(torch.from_numpy(x).to(dev), lags, spacing=61.03515625, axis=1).cpu().numpy()
    ref = post.allan(x, lags, spacing=61.03515625)
    rel_close(got, ref, 1e-10)
    # normalised, and a series length that is not a whole number of 4096-point chunks
    y = torch.from_numpy(x[:, :100000].copy()).to(dev)
    got = pk.allan(y, lags, spacing=61.03515625, normalize=True, axis=1).cpu().numpy()
    rel_close(got, post.allan(x[:, :100000], lags, spacing=61.03515625, normalize=True), 1e-10)


def test_post_reductions_are_deterministic(env):
    torch, pk, dev = env
    x = torch.from_numpy(spectra(4, 131072, 5)).to(dev)
    a = [pk.channel_average(x, 32)[0], pk.band_stats(x), pk.allan(x, [1, 8], axis=1), pk.bandpass_fit(x[0])]
    b = [pk.channel_average(x, 32)[0], pk.band_stats(x), pk.allan(x, [1, 8], axis=1), pk.bandpass_fit(x[0])]
    torch.cuda.synchronize(dev)
    for u, v in zip(a, b):
        assert torch.equal(torch.nan_to_num(u), torch.nan_to_num(v))
