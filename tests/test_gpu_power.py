"""Level histograms and total power on the GPU (counted inside the column pass) against the oracle:
counts bit-exact, power estimates to FP64 rounding (both sides evaluate the same sums and erfinv)."""
import sys

import numpy as np
import pytest

import oracle
import synth

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


def run(env, d, calls=1, hist=True):
    torch, pk, dev = env
    plan = pk.Plan([pk.Instance.from_synth(d)], device=dev)
    if hist:
        plan.set_histograms(True)
    packed = torch.from_numpy(d["packed"]).to(dev)
    plan.reset()
    per = d["n_frames"] // calls * d["fft_len"] * d["n_streams"] * d["bits"] // 8
    for c in range(calls):
        plan.accumulate(packed[c * per:packed.numel() if c == calls - 1 else (c + 1) * per])
    spec = plan.spectra()[0].cpu().numpy()
    if not hist:
        return spec, None, None, 0
    counts, power, nf = plan.histograms()
    return spec, counts.cpu().numpy(), power.cpu().numpy(), nf


@pytest.mark.parametrize("bits,log2n,F", [(2, 12, 9), (4, 14, 5), (8, 16, 6), (2, 18, 3), (8, 18, 3)])
def test_two_streams(env, bits, log2n, F):
    say(f"histograms bits={bits} N=2^{log2n} F={F}")
    d = synth.make_correlated_noise(bits, 0.3, 1 << log2n, F, seed_extra=log2n + bits)
    spec, counts, power, nf = run(env, d, calls=2 if F > 3 else 1)
    ref = oracle.level_histograms(d["packed"], bits, 2, d["n_samples"], d["pairs"])
    assert nf == F
    assert np.array_equal(counts, ref)
    pref = oracle.total_power(ref, bits)
    assert np.allclose(power[..., 0], pref[..., 0], rtol=1e-13, atol=0)
    if bits == 2:
        assert np.allclose(power[..., 1], pref[..., 1], rtol=1e-12, atol=0)
    else:
        assert np.all(np.isnan(power[..., 1]))
    # counting does not change the spectra: bitwise where both runs take the four-step passes; transforms of
    # 2^12 points or less run the single pass when not counting, equal within FP32 rounding
    spec_off = run(env, d, calls=2 if F > 3 else 1, hist=False)[0]
    if log2n > 12:
        assert np.array_equal(spec, spec_off)
    else:
        scale = np.mean(spec_off[:, 0:1, :], axis=2, keepdims=True)
        assert np.max(np.abs(spec - spec_off) / scale) < 2e-6


def test_four_streams_two_pairs(env):
    say("histograms 4 int8 streams, pairs (0,2), (1,3)")
    d = synth.make_precision(n_frames=2, fft_len=1 << 14)
    spec, counts, power, nf = run(env, d)
    ref = oracle.level_histograms(d["packed"], 8, 4, d["n_samples"], d["pairs"])
    assert np.array_equal(counts, ref)


def test_reset_and_errors(env):
    torch, pk, dev = env
    say("histogram state and errors")
    d = synth.make_correlated_noise(2, 0.1, 1 << 12, 4, seed_extra=77)
    plan = pk.Plan([pk.Instance.from_synth(d)], device=dev)
    packed = torch.from_numpy(d["packed"]).to(dev)
    with pytest.raises(pk.PolarisError) as e:
        plan.histograms()
    assert e.value.code == "PS_ERR_STATE"
    plan.set_histograms(True)
    plan.reset()
    plan.accumulate(packed)
    plan.accumulate(packed)
    c2 = plan.histograms()[0].cpu().numpy()
    plan.reset()
    plan.accumulate(packed)
    c1, _, nf = plan.histograms()
    assert nf == 4 and np.array_equal(2 * c1.cpu().numpy(), c2)
    with pytest.raises(pk.PolarisError) as e:
        plan.set_histograms(False)  # inside an integration
    assert e.value.code == "PS_ERR_STATE"
    f32 = pk.Plan([pk.Instance(fft_len=1 << 12, bits=32)], device=dev)
    with pytest.raises(pk.PolarisError) as e:
        f32.set_histograms(True)
    assert e.value.code == "PS_ERR_UNSUPPORTED"
