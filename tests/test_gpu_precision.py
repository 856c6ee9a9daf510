"""Precision form on the GPU (16-bit passes on the matrix cores) against the FP64 oracle, through the C ABI.

Error measure per Stokes product P (after Eq. 2, no fitted correction): max_k |P_gpu - P_ref| / I_ref,k.

Tolerances.  Each value is rounded to the 16-bit format three times on its way through the transform (after
the first column stage, into the inter-pass buffer, after the first row stage), with unit roundoff
u = 2^-11 (FP16) or 2^-8 (BF16); the DFT matrices carry hi + lo parts, so their own error is of order u^2.
Per frame a channel's power then has a relative error of a few u, with random sign from frame to frame, so
an integration of F frames averages it down by about 1/sqrt(F); the maximum over 2^17 channels is about 4.5
times the rms.  This gives about 3e-4 (FP16) and 2.5e-3 (BF16) at F = 32.  Bounds: FP16 1e-3 for F >= 32
(the precision form's stated tolerance); BF16 8x that (the ratio of the two roundoffs), 8e-3 for F >= 32.
Unpacking and the FP64 integration are unchanged from the plain path.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"fp16": 1e-3, "bf16": 8e-3}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1412_1256_amd as pk
    pk.lib()
    return torch, pk, torch.device("cuda:0")


def run_gpu(env, inst, precision, accum, chunk=0, calls=1):
    torch, pk, dev = env
    plan = pk.Plan([pk.Instance.from_synth(inst, precision=precision, accum=accum, chunk_frames=chunk)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.reset()
    if calls == 1:
        plan.accumulate(packed)
    else:
        per = inst["n_frames"] // calls * inst["fft_len"] * inst["n_streams"] * inst["bits"] // 8
        for c in range(calls):
            end = packed.numel() if c == calls - 1 else (c + 1) * per
            plan.accumulate(packed[c * per:end])
    st = plan.stokes()
    torch.cuda.synchronize(dev)
    return st.cpu().numpy().astype(np.float64)


def ref_stokes(inst):
    acc, nf, s2, _ = oracle.run_instance(inst)
    return oracle.stokes(acc, nf, s2)


def stokes_err(got, ref):
    I = ref[:, 0:1, :]
    return np.max(np.abs(got - ref) / I, axis=2)


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
@pytest.mark.parametrize("accum", ["fp64", "kahan32"])
@pytest.mark.parametrize("log2n", [16, 17, 18])
def test_two_stream_int8(env, precision, accum, log2n):
    say(f"precision {precision} {accum} int8 S=2 N=2^{log2n} F=32")
    inst = synth.make_correlated_noise(8, 0.3, 1 << log2n, 32, seed_extra=log2n)
    ref = ref_stokes(inst)
    got = run_gpu(env, inst, precision, accum)
    e = stokes_err(got, ref)
    say(f"  err I,Q,U,V {e.tolist()}")
    assert np.all(e < TOL[precision])


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_four_streams_two_pairs(env, precision):
    say(f"precision {precision} S=4 pairs (0,2),(1,3) N=2^18 F=48")
    inst = synth.make_precision(n_frames=48)
    ref = ref_stokes(inst)
    got = run_gpu(env, inst, precision, "kahan32")
    e = stokes_err(got, ref)
    say(f"  err per pair, I,Q,U,V {e.tolist()}")
    assert np.all(e < TOL[precision])


@pytest.mark.parametrize("pairs", [((0, 1), (2, 3)), ((3, 1),)])
def test_four_streams_other_pairs(env, pairs):
    """Four int8 streams paired otherwise than (0, 2), (1, 3): each workgroup transforms one pair, taking its
    two streams out of the four-stream word (the (0, 2), (1, 3) layout is transformed two pairs at a time)."""
    say(f"precision fp16 S=4 pairs {pairs} N=2^17 F=96")
    inst = dict(synth.make_precision(n_frames=48), pairs=[list(p) for p in pairs])
    inst = dict(inst, fft_len=1 << 17, n_frames=96)  # the same samples as 2^17-point frames
    ref = ref_stokes(inst)
    got = run_gpu(env, inst, "fp16", "kahan32")
    e = stokes_err(got, ref)
    say(f"  err per pair, I,Q,U,V {e.tolist()}")
    assert np.all(e < TOL["fp16"])


@pytest.mark.parametrize("bits", [2, 4, 32])
def test_other_formats_and_hann(env, bits):
    say(f"precision fp16 bits={bits} Hann N=2^16 F=40")
    inst = synth.make_correlated_noise(bits, 0.2, 1 << 16, 40, seed_extra=bits, window="hann")
    ref = ref_stokes(inst)
    got = run_gpu(env, inst, "fp16", "kahan32")
    e = stokes_err(got, ref)
    say(f"  err I,Q,U,V {e.tolist()}")
    assert np.all(e < TOL["fp16"])


def test_tone_dynamic_range(env):
    """A tone 40 dB above the noise per channel.  The 16-bit rounding of the column pass output scales with
    the tone in the tone's row of the inter-pass buffer, so the channels of that row carry errors relative to
    the tone rather than to their own noise: judged as spurious-free range, max_k |P_gpu - P_ref| over the
    tone's power over every other channel (bound 1e-5, i.e. spurs at least 50 dB below the tone), plus the
    tone channel itself (relative bound of the precision form)."""
    say("precision fp16 tone +40 dB S=4 N=2^18 F=32")
    inst = synth.make_precision(n_frames=32, tone_db=40.0)
    ref = ref_stokes(inst)
    got = run_gpu(env, inst, "fp16", "kahan32")
    k = 43690
    peak = ref[:, 0, k][:, None]
    assert np.all(ref[:, 0, k] > 1e3 * np.median(ref[:, 0, :], axis=1))
    d = np.abs(got - ref)
    d[:, :, k - 1:k + 2] = 0.0  # the tone's own channels are judged below
    sf = np.max(d, axis=2) / peak
    say(f"  max spur / tone per pair {sf.tolist()}")
    assert np.all(sf < 1e-5)
    et = np.abs(got[:, :, k] - ref[:, :, k]) / peak
    say(f"  tone channel err {et.tolist()}")
    assert np.all(et < TOL["fp16"])


def test_chunks_and_calls(env):
    """Frames split into chunks and over calls: same result within the rounding of the FP64 sums."""
    say("precision fp16 chunked 8 frames, 3 calls")
    inst = synth.make_correlated_noise(8, 0.3, 1 << 17, 36, seed_extra=5)
    a = run_gpu(env, inst, "fp16", "kahan32")
    b = run_gpu(env, inst, "fp16", "kahan32", chunk=8, calls=3)
    c = run_gpu(env, inst, "fp16", "kahan32")
    assert np.array_equal(a, c)  # deterministic
    rel = np.max(np.abs(a - b) / a[:, 0:1, :])
    say(f"  chunked vs whole {rel}")
    assert rel < 1e-6


@pytest.fixture(scope="module")
def config3():
    """The precision case at its stated length: 4 int8 streams (2 bands x 2 pols), 2^18 points, 610 frames
    (10 s), and its FP64 oracle Stokes."""
    inst = synth.make_precision(n_frames=610)
    return inst, ref_stokes(inst)


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_precision_config_610_frames(env, config3, precision):
    """Both 16-bit formats with Kahan-compensated integration over the 610 frames: every Stokes product of
    both pairs within 1e-3 of the oracle (per channel, relative to I).  By the estimate above the errors at
    F = 610 are about 6.9e-5 (FP16) and 5.7e-4 (BF16), the 32-frame figures times sqrt(32 / 610)."""
    inst, ref = config3
    say(f"precision case, 610 frames, {precision} + kahan32")
    got = run_gpu(env, inst, precision, "kahan32")
    e = np.max(np.abs(got - ref) / ref[:, 0:1, :], axis=2)
    say(f"  per-Stokes errors {e.tolist()}")
    assert np.all(e < 1e-3), e
