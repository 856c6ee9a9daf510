"""Overlapped segmentation and the apodisation windows on the GPU against the FP64 oracle, through the C ABI
(Sec. 3.1: frames with 50 % overlap; Hanning, Hamming and Blackman windows).

Frame f of the stream starts at sample f * hop.  Frames that span two ps_accumulate calls are transformed from
the samples the plan keeps between calls, so an integration split over calls must equal the one-call result
bit for bit (FP32 passes).  Tolerances as in the plain parity tests: per Stokes product
max_k |P_gpu - P_ref| / I_ref,k <= 1e-5 (FP32 passes), 1e-3 (FP16 passes); histograms bit-exact.
"""
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
def env():
    import torch
    import paper_1412_1256_amd as pk
    pk.lib()
    return torch, pk, torch.device("cuda:0")


def stokes_err(got, ref):
    return np.max(np.abs(got - ref) / ref[:, 0:1, :], axis=2)


def with_hop(inst, hop, window=None):
    d = dict(inst)
    d["hop"] = hop
    if window:
        d["window"] = window
    return d


def split_bytes(inst, calls):
    """Byte ranges of `calls` pieces of whole frames (the last takes the rest)."""
    N, S, b = inst["fft_len"], inst["n_streams"], inst["bits"]
    F = inst["n_samples"] // N
    per = max(1, F // calls)
    cuts = [min(F, c * per) for c in range(calls)] + [F]
    return [(cuts[c] * N * S * b // 8, cuts[c + 1] * N * S * b // 8) for c in range(calls)]


def run(env, inst, calls=1, plan=None, **over):
    torch, pk, dev = env
    plan = plan or pk.Plan([pk.Instance.from_synth(inst, **over)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.reset()
    for a, b in split_bytes(inst, calls):
        plan.accumulate(packed[a:b])
    spec, nf = plan.spectra()
    st = plan.stokes()
    torch.cuda.synchronize(dev)
    return spec.cpu().numpy(), nf, st.cpu().numpy().astype(np.float64)


def ref_stokes(inst):
    acc, nf, s2, _ = oracle.run_instance(inst)
    return oracle.stokes(acc, nf, s2), nf


@pytest.mark.parametrize("log2n,hop_div,window,bits", [
    (14, 2, "hamming", 8), (14, 4, "blackman", 2), (12, 8, "hann", 4), (16, 2, "rect", 8), (10, 2, "blackman", 32)])
def test_overlapped_frames_against_oracle(env, log2n, hop_div, window, bits):
    N = 1 << log2n
    inst = with_hop(synth.make_correlated_noise(bits, 0.3, N, 40, seed_extra=log2n + hop_div, window=window),
                    N // hop_div)
    say(f"overlap N=2^{log2n} hop=N/{hop_div} {window} bits={bits}")
    ref, nf_ref = ref_stokes(inst)
    _, nf, got = run(env, inst)
    assert nf == nf_ref == hop_div * 40 - (hop_div - 1)
    e = stokes_err(got, ref)
    say(f"  frames {nf} err {e.tolist()}")
    assert np.all(e < TOL)


@pytest.mark.parametrize("hop_div,calls,chunk", [(2, 3, 0), (4, 5, 0), (2, 7, 3)])
def test_split_calls_bitwise_equal_one_call(env, hop_div, calls, chunk):
    N = 1 << 13
    inst = with_hop(synth.make_correlated_noise(8, 0.25, N, 21, seed_extra=hop_div * 10 + calls, window="hamming"),
                    N // hop_div)
    say(f"overlap split calls hop=N/{hop_div} calls={calls} chunk={chunk}")
    s1, n1, t1 = run(env, inst, calls=1, chunk_frames=chunk)
    s2, n2, t2 = run(env, inst, calls=calls, chunk_frames=chunk)
    assert n1 == n2 == hop_div * 21 - (hop_div - 1)
    assert np.array_equal(s1, s2)
    assert np.array_equal(t1, t2)


def test_paper_size_half_overlap(env):
    """2^18-point frames, 50 % overlap, Hamming window, int8 two streams, over two calls."""
    N = 1 << 18
    inst = with_hop(synth.make_correlated_noise(8, 0.3, N, 8, seed_extra=18, window="hamming"), N // 2)
    say("overlap N=2^18 hop=N/2 hamming int8 two calls")
    ref, nf_ref = ref_stokes(inst)
    _, nf, got = run(env, inst, calls=2)
    assert nf == nf_ref == 15
    e = stokes_err(got, ref)
    say(f"  err {e.tolist()}")
    assert np.all(e < TOL)


def test_grouped_plan_with_overlap_equals_separate_plans(env):
    torch, pk, dev = env
    insts = [with_hop(synth.make_correlated_noise(8, 0.2, 1 << 12, 30, seed_extra=1), 1 << 11),
             synth.make_correlated_noise(2, 0.3, 1 << 12, 20, seed_extra=2),
             with_hop(synth.make_correlated_noise(2, 0.4, 1 << 14, 12, seed_extra=3, window="blackman"), 1 << 12),
             with_hop(synth.make_mode("4MHz", n_frames=6), 1 << 16),
             synth.make_mode("8MHz", n_frames=4)]
    say("grouped plan of overlapped and contiguous instances (two and four streams), two calls")
    plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev)
    bufs = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
    plan.reset()
    for c in range(2):
        pieces = [b[slice(*split_bytes(d, 2)[c])] for d, b in zip(insts, bufs)]
        plan.accumulate(pieces)
    grouped = [plan.spectra(i)[0].cpu().numpy() for i in range(len(insts))]
    for i, d in enumerate(insts):
        sep = run(env, d, calls=2)[0]
        assert np.array_equal(grouped[i], sep), i


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_precision_form_with_overlap(env, precision):
    N = 1 << 16
    inst = with_hop(synth.make_correlated_noise(8, 0.3, N, 17, seed_extra=60, window="blackman"), N // 2)
    say(f"overlap precision {precision} N=2^16 hop=N/2 blackman")
    ref, _ = ref_stokes(inst)
    _, nf, got = run(env, inst, calls=2, precision=precision, accum="kahan32")
    assert nf == 33
    e = stokes_err(got, ref)
    say(f"  err {e.tolist()}")
    assert np.all(e < {"fp16": 1e-3, "bf16": 8e-3}[precision])


@pytest.mark.parametrize("bits,hop_div", [(2, 2), (8, 4), (4, 2)])
def test_histograms_count_every_sample_once(env, bits, hop_div):
    torch, pk, dev = env
    N = 1 << 12
    inst = with_hop(synth.make_correlated_noise(bits, 0.3, N, 9, seed_extra=bits), N // hop_div)
    say(f"overlap histograms bits={bits} hop=N/{hop_div} three calls")
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    plan.set_histograms(True)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.reset()
    for a, b in split_bytes(inst, 3):
        plan.accumulate(packed[a:b])
    counts, _, nf = plan.histograms()
    counts = counts.cpu().numpy()
    hop = N // hop_div
    counted = inst["n_samples"] - (N - hop)  # the last N - hop samples wait for a next call
    ref = oracle.level_histograms(inst["packed"][:counted * 2 * bits // 8], bits, 2, counted, inst["pairs"])
    assert nf == hop_div * 9 - (hop_div - 1)
    assert np.array_equal(counts, ref)


def test_state_export_import_carries_waiting_samples(env):
    torch, pk, dev = env
    N = 1 << 12
    inst = with_hop(synth.make_correlated_noise(8, 0.3, N, 12, seed_extra=44, window="hann"), N // 2)
    say("overlap state export/import between calls")
    packed = torch.from_numpy(inst["packed"]).to(dev)
    (a0, b0), (a1, b1) = split_bytes(inst, 2)
    p1 = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    p1.reset()
    p1.accumulate(packed[a0:b0])
    state, nf = p1.state_export()
    p2 = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    p2.reset()
    p2.state_import(state, nf)
    p2.accumulate(packed[a1:b1])
    p1.accumulate(packed[a1:b1])
    s1, n1 = p1.spectra()
    s2, n2 = p2.spectra()
    torch.cuda.synchronize(dev)
    assert n1 == n2 == 23
    assert torch.equal(s1, s2)


def test_graph_replay_with_overlap(env):
    torch, pk, dev = env
    N = 1 << 13
    inst = with_hop(synth.make_correlated_noise(8, 0.3, N, 10, seed_extra=45, window="hamming"), N // 4)
    say("overlap graph capture of a two-call integration")
    side = torch.cuda.Stream(dev)
    with torch.cuda.stream(side):
        plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev, stream=side)
        packed = torch.from_numpy(inst["packed"]).to(dev)
        out = torch.zeros((1, 4, N // 2), dtype=torch.float32, device=dev)
    side.synchronize()
    (a0, b0), (a1, b1) = split_bytes(inst, 2)

    def integration():
        plan.reset()
        plan.accumulate(packed[a0:b0])
        plan.accumulate(packed[a1:b1])
        plan.stokes(out=out)

    with torch.cuda.stream(side):
        integration()
    side.synchronize()
    eager = out.clone()
    plan.graph_capture(integration)
    for r in range(3):
        out.zero_()
        torch.cuda.synchronize(dev)
        plan.graph_replay()
        side.synchronize()
        assert torch.equal(out, eager), r
        _ = (packed[:1024].float() * 2).sum().item()  # eager work between replays


def test_overlapped_taps_gradient(env):
    """The window adjoint with overlapped frames (each sample in two frames at two window positions)."""
    torch, pk, dev = env
    N, F = 1 << 12, 10
    rng = np.random.default_rng(77)
    inst = with_hop(synth.make_correlated_noise(8, 0.3, N, F, seed_extra=77, window="taps"), N // 2)
    taps = (1 + 0.1 * rng.standard_normal(64)).astype(np.float32)
    g = rng.standard_normal((1, 4, N // 2)).astype(np.float32)
    say("overlap window-tap gradient hop=N/2")
    w, s2 = oracle.window("taps", N, taps=taps.astype(np.float64))
    acc, nf = oracle.accumulate(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"], hop=N // 2)
    gr = oracle.calibrate_backward(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"], acc, nf, s2,
                                   g.astype(np.float64), taps=taps.astype(np.float64), hop=N // 2)
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.set_window_taps(torch.from_numpy(taps).to(dev))
    plan.reset()
    plan.accumulate(packed)
    grads = plan.calibrate_backward(packed, torch.from_numpy(g).to(dev), want=("taps",))
    torch.cuda.synchronize(dev)
    dt = grads["taps"].cpu().numpy().astype(np.float64)
    rel = np.max(np.abs(dt - gr["d_taps"])) / np.max(np.abs(gr["d_taps"]))
    say(f"  frames {nf} taps rel err {rel}")
    assert nf == 2 * F - 1
    assert rel < 1e-4
