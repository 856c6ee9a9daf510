"""Single-pass short transforms (whole frames in LDS, N = 2^8 .. 2^12) on the GPU against the FP64 oracle and
against the four-step passes, through the C ABI.

Bounds as in the plain parity tests: per Stokes product max_k |P_gpu - P_ref| / I_ref,k <= 1e-5 (>= 32
frames); spectra normwise max_k |d| / mean_k XX_ref <= 1e-5.  Single pass vs four-step: the same
quantities within FP32 rounding of the two transforms (normwise 2e-6).  Split calls and repeated runs:
bitwise equal.
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


def spectra_err(got, ref):
    return np.max(np.abs(got - ref) / np.mean(ref[:, 0:1, :], axis=2, keepdims=True), axis=2)


def run(env, inst, sched=None, calls=1, psi=0.0):
    torch, pk, dev = env
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev, schedules=None if sched is None else [sched])
    packed = torch.from_numpy(inst["packed"]).to(dev)
    N, S, b = inst["fft_len"], inst["n_streams"], inst["bits"]
    F = inst["n_samples"] // N
    per = max(1, F // calls)
    cuts = [min(F, c * per) for c in range(calls)] + [F]
    plan.reset()
    for c in range(calls):
        plan.accumulate(packed[cuts[c] * N * S * b // 8:cuts[c + 1] * N * S * b // 8])
    spec, nf = plan.spectra()
    st = plan.stokes(psi=psi)
    torch.cuda.synchronize(dev)
    return spec.cpu().numpy(), nf, st.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("log2n", [8, 9, 10, 11, 12])
@pytest.mark.parametrize("bits,window", [(2, "rect"), (4, "hann"), (8, "hamming"), (32, "blackman")])
def test_single_pass_against_oracle(env, log2n, bits, window):
    torch, pk, dev = env
    inst = synth.make_correlated_noise(bits, 0.3, 1 << log2n, 40, seed_extra=log2n * 10 + bits, window=window)
    say(f"single pass N=2^{log2n} bits={bits} {window}")
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2, psi=0.2)
    spec, gnf, st = run(env, inst, psi=0.2)
    assert gnf == nf == 40
    es, e = spectra_err(spec, acc), stokes_err(st, ref)
    say(f"  spectra {es.max()} stokes {e.tolist()}")
    assert np.all(es < TOL) and np.all(e < TOL)


@pytest.mark.parametrize("bits", [2, 8])
def test_four_streams_two_pairs(env, bits):
    torch, pk, dev = env
    rng = synth.rng_for(300, bits)
    N, F = 4096, 36
    base = rng.standard_normal((4, N * F))
    x = np.stack([base[0], base[1], 0.6 * base[0] + 0.8 * base[2], 0.3 * base[1] + 0.95 * base[3]], axis=1)
    if bits == 8:
        x = x * 16
    inst = dict(packed=synth.pack_codes(synth.quantize(x, bits), bits), bits=bits, n_streams=4, fft_len=N,
                n_frames=F, n_samples=N * F, window="rect", pairs=[(0, 2), (1, 3)])
    say(f"single pass four streams bits={bits}")
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2)
    spec, gnf, st = run(env, inst)
    assert np.all(stokes_err(st, ref) < TOL)


@pytest.mark.parametrize("log2n", [8, 10, 12])
def test_single_pass_matches_four_step(env, log2n):
    torch, pk, dev = env
    inst = synth.make_correlated_noise(8, 0.3, 1 << log2n, 64, seed_extra=log2n, window="hann")
    say(f"single pass vs four-step N=2^{log2n}")
    a, _, _ = run(env, inst)
    b, _, _ = run(env, inst, sched=pk.Schedule(single_pass=2))
    e = spectra_err(a, b)
    say(f"  {e.max()}")
    assert e.max() < 2e-6


@pytest.mark.parametrize("slots", [1, 4, 64, 1024])
def test_slot_counts_and_split_calls(env, slots):
    torch, pk, dev = env
    inst = synth.make_correlated_noise(8, 0.25, 2048, 150, seed_extra=slots)
    sched = pk.Schedule(rowpass_slots=slots, single_pass=1)
    say(f"single pass G={slots} split calls")
    a, n1, _ = run(env, inst, sched=sched)
    b, n2, _ = run(env, inst, sched=sched, calls=4)
    c, _, _ = run(env, inst, sched=sched)
    assert n1 == n2 == 150
    assert np.array_equal(a, b) and np.array_equal(a, c)
    acc, nf, s2, _ = oracle.run_instance(inst)
    assert np.all(spectra_err(a, acc) < TOL)


def test_overlap_and_histograms(env):
    """50 % overlap through the single pass over three calls; an integration with level histograms on runs
    the four-step column pass, which counts, for the same instance."""
    torch, pk, dev = env
    N = 1024
    inst = dict(synth.make_correlated_noise(2, 0.3, N, 30, seed_extra=77, window="hann"), hop=N // 2)
    say("single pass with overlap; histograms")
    acc, nf, s2, _ = oracle.run_instance(inst)
    spec, gnf, _ = run(env, inst, calls=3)
    assert gnf == nf == 59
    assert np.all(spectra_err(spec, acc) < TOL)
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    half = packed.numel() // 2
    plan.reset()
    plan.set_histograms(True)
    plan.accumulate(packed[:half])
    plan.accumulate(packed[half:])
    spec2, nf2 = plan.spectra()
    counts, _, _ = plan.histograms()
    torch.cuda.synchronize(dev)
    assert nf2 == 59
    assert np.all(spectra_err(spec2.cpu().numpy(), acc) < TOL)
    counted = inst["n_samples"] - N // 2  # the last N - hop samples wait for a next call
    ref = oracle.level_histograms(inst["packed"][:counted * 2 * 2 // 8], 2, 2, counted, inst["pairs"])
    assert np.array_equal(counts.cpu().numpy(), ref)


def test_state_graph_and_grouped_plans(env):
    torch, pk, dev = env
    insts = [synth.make_correlated_noise(8, 0.2, 4096, 50, seed_extra=1),
             synth.make_correlated_noise(2, 0.3, 1 << 16, 6, seed_extra=2),
             synth.make_correlated_noise(4, 0.4, 512, 200, seed_extra=3, window="hann")]
    say("single pass: grouped plan, state export/import, graph replay")
    packed = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
    side = torch.cuda.Stream(dev)
    with torch.cuda.stream(side):
        plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev, stream=side)
        outs = [torch.zeros((1, 4, d["fft_len"] // 2), dtype=torch.float32, device=dev) for d in insts]
    side.synchronize()

    def integration():
        plan.reset()
        plan.accumulate(packed)
        plan.stokes_all(outs)

    with torch.cuda.stream(side):
        integration()
    side.synchronize()
    eager = [o.clone() for o in outs]
    for i, d in enumerate(insts):
        one = pk.Plan([pk.Instance.from_synth(d)], device=dev)
        one.reset()
        one.accumulate(packed[i])
        assert torch.equal(one.stokes(), eager[i]), i
        # export after the first half, import into a fresh plan, finish there
        h = packed[i].numel() // 2
        one.reset()
        one.accumulate(packed[i][:h])
        state, nf = one.state_export()
        two = pk.Plan([pk.Instance.from_synth(d)], device=dev)
        two.reset()
        two.state_import(state, nf)
        two.accumulate(packed[i][h:])
        assert torch.equal(two.stokes(), eager[i]), i
    plan.graph_capture(integration)
    for r in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize(dev)
        plan.graph_replay()
        side.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), r


def test_backward_reads_reduced_slots(env):
    """More than 64 slots in use: Stokes and the adjoint read the reduced slot sum (learnable window)."""
    torch, pk, dev = env
    N, F = 1024, 200
    rng = np.random.default_rng(8)
    inst = synth.make_correlated_noise(8, 0.3, N, F, seed_extra=8, window="taps")
    taps = (1 + 0.1 * rng.standard_normal(64)).astype(np.float32)
    g = rng.standard_normal((1, 4, N // 2)).astype(np.float32)
    say("single pass backward with 200 slots in use")
    w, s2 = oracle.window("taps", N, taps=taps.astype(np.float64))
    acc, nf = oracle.accumulate(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"])
    ref = oracle.stokes(acc, nf, s2)
    gr = oracle.calibrate_backward(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"], acc, nf, s2,
                                   g.astype(np.float64), taps=taps.astype(np.float64))
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.set_window_taps(torch.from_numpy(taps).to(dev))
    plan.reset()
    plan.accumulate(packed)
    st = plan.stokes().cpu().numpy().astype(np.float64)
    grads = plan.calibrate_backward(packed, torch.from_numpy(g).to(dev))
    torch.cuda.synchronize(dev)
    assert np.all(stokes_err(st, ref) < TOL)
    for name, key in (("gain_x", "d_gain_x"), ("gain_y", "d_gain_y")):
        got = grads[name].cpu().numpy().astype(np.float64)
        got = got[..., 0] + 1j * got[..., 1]
        rel = np.max(np.abs(got - gr[key])) / np.max(np.abs(gr[key]))
        assert rel < 1e-5, (name, rel)
    dt = grads["taps"].cpu().numpy().astype(np.float64)
    rel = np.max(np.abs(dt - gr["d_taps"])) / np.max(np.abs(gr["d_taps"]))
    say(f"  taps rel err {rel}")
    assert rel < 1e-4
