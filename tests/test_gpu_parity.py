"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (FP32 passes, FP64 accumulation):
  * unpack: bit-exact;
  * Stokes: max_k |P_gpu - P_ref| / I_ref,k <= 1e-5 for each of I, Q, U, V (integrations of >= 32 frames, where
    every channel's I is far from zero);
  * spectra of short integrations: max_k |d| / mean_k(XX_ref) <= 1e-5 (normwise; single channels of a 1-frame
    noise spectrum can be arbitrarily close to zero, so a per-channel relative bound does not apply).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def pk():
    import paper_1412_1256_amd as pk
    pk.lib()
    return pk


def run_gpu(pk, torch, dev, inst, psi=0.0, gains=None, dterms=None, chunk=0):
    plan = pk.Plan([pk.Instance.from_synth(inst, chunk_frames=chunk)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.reset()
    plan.accumulate(packed)
    spec, nf = plan.spectra()
    gx = gy = None
    if gains is not None:
        gx = torch.from_numpy(np.ascontiguousarray(gains[0])).to(dev)
        gy = torch.from_numpy(np.ascontiguousarray(gains[1])).to(dev)
    dt = None if dterms is None else torch.from_numpy(np.ascontiguousarray(dterms)).to(dev)
    st = plan.stokes(psi=psi, gain_x=gx, gain_y=gy, dterms=dt)
    torch.cuda.synchronize(dev)
    return spec.cpu().numpy(), nf, st.cpu().numpy().astype(np.float64)


def stokes_err(got, ref):
    """per pair and product: max_k |got - ref| / I_ref,k"""
    I = ref[:, 0:1, :]
    return np.max(np.abs(got - ref) / I, axis=2)


def spectra_err(got, ref):
    """per pair and product: max_k |got - ref| / mean_k XX_ref"""
    scale = np.mean(ref[:, 0:1, :], axis=2, keepdims=True)
    return np.max(np.abs(got - ref) / scale, axis=2)


# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("bits,S,n_time", [(2, 2, 4096 + 6), (4, 2, 999), (8, 2, 70001), (32, 2, 513),
                                           (2, 4, 1030), (8, 4, 777), (4, 1, 8), (8, 8, 123)])
def test_unpack_bit_exact(pk, torch_dev, bits, S, n_time):
    torch, dev = torch_dev
    say(f"unpack bits={bits} S={S} n_time={n_time}")
    rng = np.random.default_rng(bits * 100 + S)
    nbytes = (n_time * S * bits + 7) // 8
    if bits == 32:
        raw = rng.standard_normal(n_time * S).astype(np.float32).view(np.uint8)
    else:
        raw = rng.integers(0, 256, nbytes, dtype=np.uint8)
    ref = oracle.unpack(raw, bits, S, n_time).astype(np.float32)
    got = pk.unpack(torch.from_numpy(raw).to(dev), bits, S, n_time).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_tiny_config(pk, torch_dev):
    """2 x 2-bit streams, rho = 0.3, tone at channel 100, 1024-point Hann frames, 64 frames."""
    torch, dev = torch_dev
    say("tiny config")
    inst = synth.make_tiny()
    acc, nf, s2, _ = oracle.run_instance(inst)
    for psi in (0.0, 0.4):
        ref = oracle.stokes(acc, nf, s2, psi=psi)
        spec, gnf, st = run_gpu(pk, torch, dev, inst, psi=psi)
        assert gnf == nf == 64
        e = stokes_err(st, ref)
        say(f"  psi={psi} stokes err {e.tolist()}")
        assert np.all(e < TOL), e
        assert np.all(spectra_err(spec, acc) < TOL)


@pytest.mark.parametrize("logn", list(range(8, 21)))
def test_fft_lengths_float_input(pk, torch_dev, logn):
    """Float32 correlated noise, Hann window, 3 frames (a ragged frame batch), every supported length."""
    torch, dev = torch_dev
    N = 1 << logn
    say(f"fft length 2^{logn}")
    inst = synth.make_correlated_noise(32, 0.4, N, 3, seed_extra=logn, window="hann")
    acc, nf, s2, _ = oracle.run_instance(inst)
    spec, gnf, st = run_gpu(pk, torch, dev, inst)
    assert gnf == 3
    e = spectra_err(spec, acc)
    say(f"  spectra err {e.ravel().tolist()}")
    assert np.all(e < TOL), e


@pytest.mark.parametrize("logn,F", [(13, 300), (14, 150), (15, 80), (16, 48), (17, 40), (19, 40), (20, 32)])
def test_default_schedules_many_frames(pk, torch_dev, logn, F):
    """2-bit pair, Hann window, the default schedules of 2^13 .. 2^17 points (longer column pass first,
    several column-pass workgroups per CU, row-pass slots aimed at 512 workgroups), of 2^19 (1024 x 512,
    4-frame row batches) and 2^20 (512 x 2048) over enough frames that every frame group and slot is used;
    one call against the oracle, three calls bitwise equal to one."""
    torch, dev = torch_dev
    N = 1 << logn
    say(f"default schedule 2^{logn}, {F} frames")
    inst = synth.make_correlated_noise(2, 0.35, N, F, seed_extra=500 + logn, window="hann")
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2, psi=0.3)
    spec, gnf, st = run_gpu(pk, torch, dev, inst, psi=0.3)
    assert gnf == nf == F
    es, e = spectra_err(spec, acc), stokes_err(st, ref)
    say(f"  spectra {es.max()} stokes {e.ravel().tolist()}")
    assert np.all(es < TOL) and np.all(e < TOL), (es, e)
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    per = N * 2 * 2 // 8
    cuts = [0, (F // 3) * per, (2 * F // 3 + 1) * per, F * per]
    plan.reset()
    for c in range(3):
        plan.accumulate(packed[cuts[c]:cuts[c + 1]])
    split, nf2 = plan.spectra()
    torch.cuda.synchronize(dev)
    assert nf2 == F
    assert np.array_equal(split.cpu().numpy(), spec)


@pytest.mark.parametrize("logn", [21, 22])
def test_largest_lengths(pk, torch_dev, logn):
    torch, dev = torch_dev
    N = 1 << logn
    say(f"fft length 2^{logn} (8-bit, rect)")
    inst = synth.make_correlated_noise(8, 0.2, N, 2, seed_extra=logn)
    acc, nf, s2, _ = oracle.run_instance(inst)
    spec, gnf, st = run_gpu(pk, torch, dev, inst)
    e = spectra_err(spec, acc)
    say(f"  spectra err {e.ravel().tolist()}")
    assert np.all(e < TOL), e


def test_paper_config_full_size(pk, torch_dev):
    """2 int8 streams, 2^18 points, 61 frames, lines and Zeeman-like V: full-size parity."""
    torch, dev = torch_dev
    say("paper-shaped config, full size")
    inst = synth.make_paper()
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2, psi=0.25)
    spec, gnf, st = run_gpu(pk, torch, dev, inst, psi=0.25)
    assert gnf == nf == 61
    e = stokes_err(st, ref)
    say(f"  stokes err {e.tolist()}")
    assert np.all(e < TOL), e
    # spectra: XX, YY relative per channel; XY relative to sqrt(XX YY)
    ex = np.max(np.abs(spec[0, 0] - acc[0, 0]) / acc[0, 0])
    ey = np.max(np.abs(spec[0, 1] - acc[0, 1]) / acc[0, 1])
    exy = np.max(np.hypot(spec[0, 2] - acc[0, 2], spec[0, 3] - acc[0, 3]) / np.sqrt(acc[0, 0] * acc[0, 1]))
    say(f"  spectra err xx={ex:.3g} yy={ey:.3g} xy={exy:.3g}")
    assert max(ex, ey, exy) < TOL


@pytest.mark.parametrize("bits", [2, 4, 8])
def test_four_streams_two_pairs(pk, torch_dev, bits):
    """Table 1 layout X0, X1, Y0, Y1 with pairs (X0, Y0), (X1, Y1)."""
    torch, dev = torch_dev
    say(f"four streams bits={bits}")
    rng = synth.rng_for(200, bits)
    N, F = 4096, 40
    T = N * F
    base = rng.standard_normal((4, T))
    x = np.stack([base[0], base[1], 0.6 * base[0] + 0.8 * base[2], 0.3 * base[1] + 0.95 * base[3]], axis=1)
    if bits == 8:
        x = x * 16
    codes = synth.quantize(x, bits)
    inst = dict(packed=synth.pack_codes(codes, bits), bits=bits, n_streams=4, fft_len=N, n_frames=F,
                n_samples=T, window="rect", pairs=[(0, 2), (1, 3)])
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2)
    spec, gnf, st = run_gpu(pk, torch, dev, inst)
    e = stokes_err(st, ref)
    say(f"  stokes err {e.tolist()}")
    assert np.all(e < TOL), e


def test_calibration_gains_and_leakage(pk, torch_dev):
    torch, dev = torch_dev
    say("calibrated stokes with gains and d-terms")
    inst = synth.make_correlated_noise(8, 0.3, 2048, 40, seed_extra=5)
    rng = np.random.default_rng(8)
    C_ = 1024
    gx = (1 + 0.1 * (rng.standard_normal(C_) + 1j * rng.standard_normal(C_))).astype(np.complex64)
    gy = (1 + 0.1 * (rng.standard_normal(C_) + 1j * rng.standard_normal(C_))).astype(np.complex64)
    dt = np.array([[0.02 * np.exp(0.3j), 0.03 * np.exp(-1.3j)]], dtype=np.complex64)
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2, gain_x=gx[None].astype(np.complex128), gain_y=gy[None].astype(np.complex128),
                        dterms=dt.astype(np.complex128), psi=-0.7)
    gxr = np.ascontiguousarray(np.stack([gx.real, gx.imag], -1)[None]).astype(np.float32)
    gyr = np.ascontiguousarray(np.stack([gy.real, gy.imag], -1)[None]).astype(np.float32)
    dtr = np.array([[dt[0, 0].real, dt[0, 0].imag, dt[0, 1].real, dt[0, 1].imag]], dtype=np.float32)
    spec, gnf, st = run_gpu(pk, torch, dev, inst, psi=-0.7, gains=(gxr, gyr), dterms=dtr)
    e = stokes_err(st, ref)
    say(f"  stokes err {e.tolist()}")
    assert np.all(e < TOL), e


def test_identical_streams_cross_equals_auto(pk, torch_dev):
    torch, dev = torch_dev
    say("identical streams")
    inst = synth.make_identical_streams(8, 8192, 33)
    spec, nf, st = run_gpu(pk, torch, dev, inst)
    xx = spec[0, 0]
    assert np.max(np.abs(spec[0, 2] - xx) / xx) < TOL
    assert np.max(np.abs(spec[0, 3]) / xx) < TOL
    assert np.max(np.abs(spec[0, 1] - xx) / xx) < TOL


def test_pure_tone_lands_in_one_channel(pk, torch_dev):
    torch, dev = torch_dev
    say("pure tone")
    N, k0, A = 1 << 16, 12345, 3.0
    inst = synth.make_tone_f32(N, 2, k0, amp=A, phase=0.3, phase_y=1.1)
    spec, nf, st = run_gpu(pk, torch, dev, inst)
    peak = (A * N / 2) ** 2 * 2
    assert abs(spec[0, 0, k0] - peak) / peak < 1e-6
    others = np.delete(spec[0, 0], k0)
    assert np.max(others) < 1e-9 * peak
    # XY* phase = phase_x - phase_y
    ph = math.atan2(spec[0, 3, k0], spec[0, 2, k0])
    assert abs(ph - (0.3 - 1.1)) < 1e-5


@pytest.mark.parametrize("logn,k0", [(19, 54321), (20, 12345), (20, 512 * 700), (20, 256 + 512 * 77)])
def test_pure_tone_long_rows(pk, torch_dev, logn, k0):
    """Pure tones through the long rows (2^19: 512 x 1024, 2^20: 512 x 2048, whose rows are transformed as
    two halves of even and odd samples): the closed-form peak in channel k0 and nothing elsewhere, including
    tones on row 0 and row N1/2, where a bin pairs with its own row."""
    torch, dev = torch_dev
    say(f"pure tone 2^{logn} k0={k0}")
    N, A = 1 << logn, 3.0
    inst = synth.make_tone_f32(N, 2, k0, amp=A, phase=0.3, phase_y=1.1)
    spec, nf, st = run_gpu(pk, torch, dev, inst)
    peak = (A * N / 2) ** 2 * 2
    err = abs(spec[0, 0, k0] - peak) / peak
    others = np.delete(spec[0, 0], k0)
    say(f"  peak err {err} leakage {np.max(others) / peak}")
    assert err < 2e-6
    assert np.max(others) < 1e-9 * peak
    ph = math.atan2(spec[0, 3, k0], spec[0, 2, k0])
    assert abs(ph - (0.3 - 1.1)) < 1e-5


def test_split_calls_are_bitwise_identical(pk, torch_dev):
    torch, dev = torch_dev
    say("split calls")
    inst = synth.make_correlated_noise(8, 0.1, 4096, 23, seed_extra=2)
    N = 4096
    bpf = N * 2
    packed = torch.from_numpy(inst["packed"]).to(dev)
    whole = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    whole.reset()
    whole.accumulate(packed)
    a, _ = whole.spectra()
    split = pk.Plan([pk.Instance.from_synth(inst, chunk_frames=5)], device=dev)
    split.reset()
    for lo, hi in ((0, 7), (7, 8), (8, 23)):
        split.accumulate(packed[lo * bpf:hi * bpf])
    b, nf = split.spectra()
    torch.cuda.synchronize(dev)
    assert nf == 23
    assert torch.equal(a, b)


def test_run_to_run_determinism_and_reset(pk, torch_dev):
    torch, dev = torch_dev
    say("determinism")
    inst = synth.make_correlated_noise(2, 0.2, 1 << 14, 9, seed_extra=4)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    outs = []
    for _ in range(3):
        plan.reset()
        plan.accumulate(packed)
        outs.append(plan.spectra()[0].clone())
    torch.cuda.synchronize(dev)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[1], outs[2])


def test_state_export_import_resumes_bitwise(pk, torch_dev):
    torch, dev = torch_dev
    say("state export/import")
    inst = synth.make_correlated_noise(8, 0.3, 2048, 12, seed_extra=6)
    bpf = 2048 * 2
    packed = torch.from_numpy(inst["packed"]).to(dev)
    ref_plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    ref_plan.reset()
    ref_plan.accumulate(packed)
    ref, _ = ref_plan.spectra()
    p1 = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    p1.reset()
    p1.accumulate(packed[:5 * bpf])
    state, nf = p1.state_export()
    p2 = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    p2.state_import(state, nf)
    p2.accumulate(packed[5 * bpf:])
    got, nf2 = p2.spectra()
    torch.cuda.synchronize(dev)
    assert nf == 5 and nf2 == 12
    assert torch.equal(ref, got)


def test_error_paths(pk, torch_dev):
    torch, dev = torch_dev
    say("error paths")
    inst = synth.make_correlated_noise(8, 0.3, 1024, 2)
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.reset()
    with pytest.raises(pk.PolarisError) as e:
        plan.stokes()
    assert e.value.code == "PS_ERR_STATE"
    with pytest.raises(pk.PolarisError) as e:
        plan.accumulate(packed[:1000], n_samples=[500])
    assert e.value.code == "PS_ERR_SIZE"
    plan.accumulate(packed[:0], n_samples=[0])  # empty input is a no-op
    with pytest.raises(pk.PolarisError):
        plan.spectra()
    plan.accumulate(packed)
    s, nf = plan.spectra()
    assert nf == 2


def test_reused_input_buffer_between_calls(pk, torch_dev):
    """Streaming: one device buffer is overwritten with new sampler data before each call."""
    torch, dev = torch_dev
    say("reused input buffer")
    N, F = 1 << 18, 6
    inst = synth.make_correlated_noise(8, 0.2, N, 2 * F, seed_extra=11)
    bpc = N * 2 * F  # bytes per call
    host = torch.from_numpy(inst["packed"])
    buf = torch.empty(bpc, dtype=torch.uint8, device=dev)
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    plan.reset()
    for c in range(2):
        buf.copy_(host[c * bpc:(c + 1) * bpc].to(dev))
        plan.accumulate(buf)
    got, nf = plan.spectra()
    torch.cuda.synchronize(dev)
    acc, nfo, s2, _ = oracle.run_instance(inst)
    assert nf == nfo == 2 * F
    e = spectra_err(got.cpu().numpy(), acc)
    say(f"  spectra err {e.ravel().tolist()}")
    assert np.all(e < TOL), e


@pytest.mark.parametrize("psi", [0.0, 0.7])
def test_circular_feeds(pk, torch_dev, psi):
    """Streams taken as R, L: the circular-feed combination with gains and leakage against the oracle."""
    torch, dev = torch_dev
    say(f"circular feeds psi={psi}")
    inst = synth.make_correlated_noise(8, 0.4, 1 << 14, 40, seed_extra=90)
    rng = np.random.default_rng(90)
    C = inst["fft_len"] // 2
    gx = (1 + 0.05 * (rng.standard_normal((1, C)) + 1j * rng.standard_normal((1, C)))).astype(np.complex64)
    gy = (1 + 0.05 * (rng.standard_normal((1, C)) + 1j * rng.standard_normal((1, C)))).astype(np.complex64)
    dt = (0.02 * np.exp(1j * rng.uniform(0, 6.28, (1, 2)))).astype(np.complex64)
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2, gain_x=gx.astype(np.complex128), gain_y=gy.astype(np.complex128),
                        dterms=dt.astype(np.complex128), psi=psi, feed="circular")
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    plan.reset()
    plan.accumulate(torch.from_numpy(inst["packed"]).to(dev))
    got = plan.stokes(gain_x=torch.from_numpy(gx).to(dev), gain_y=torch.from_numpy(gy).to(dev),
                      dterms=torch.from_numpy(dt).to(dev), psi=psi, feed="circular").cpu().numpy()
    e = stokes_err(got.astype(np.float64), ref)
    say(f"  err {e.tolist()}")
    assert np.all(e < TOL)
    with pytest.raises(pk.PolarisError) as ex:
        plan.stokes(feed=5)
    assert ex.value.code == "PS_ERR_ARG"


@pytest.mark.parametrize("mode,F", [("8MHz", 16), ("4MHz", 32)])
def test_table1_modes(pk, torch_dev, mode, F):
    """Table 1's sampler modes with their four IFs: 8 MHz (16 Msps, 4-bit, 2^18 points) and 4 MHz (8 Msps,
    8-bit, 2^17 points), pairs (X0, Y0), (X1, Y1)."""
    torch, dev = torch_dev
    say(f"Table 1 mode {mode} F={F}")
    inst = synth.make_mode(mode, n_frames=F)
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2, psi=0.3)
    spec, gnf, st = run_gpu(pk, torch, dev, inst, psi=0.3)
    assert gnf == nf == F
    e_spec = spectra_err(spec, acc)
    e = stokes_err(st, ref)
    say(f"  spectra err {e_spec.max()} stokes err {e.tolist()}")
    assert np.all(e_spec < TOL) and np.all(e < TOL), (e_spec, e)
