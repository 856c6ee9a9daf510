"""Batching form on the GPU: grouped launches over many uneven instances, and hipGraph replay.

Parity: the grouped launches run the same per-tile code as single-instance plans, and the row pass adds the
frames of each instance in order, so the spectra of a many-instance plan equal those of one plan per
instance bit for bit; a few instances are also checked against the FP64 oracle (Stokes tolerance 1e-5, as
for the plain path).  Graph replays are compared with the eager result after every replay, with eager work
and synchronisations in between.
"""
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


def mixed_set():
    """Uneven instances: N = 2^8 .. 2^16, 2/4/8-bit and float, 2 or 4 streams, rect and Hann."""
    out = []
    rng = np.random.default_rng(7)
    for i, (e, F, bits) in enumerate([(8, 5, 2), (9, 17, 8), (10, 3, 8), (11, 9, 2), (12, 12, 8), (13, 8, 4),
                                      (14, 6, 8), (15, 4, 2), (16, 3, 8), (12, 1, 32), (10, 20, 8), (9, 2, 2)]):
        win = "hann" if i % 5 == 4 else "rect"
        out.append(synth.make_correlated_noise(bits, float(rng.uniform(0, 0.5)), 1 << e, F, cfg=4,
                                               seed_extra=300 + i, window=win))
    out.append(synth.make_precision(n_frames=3, fft_len=1 << 12))  # 4 streams, 2 pairs
    return out


def run(env, insts, chunk=0, separate=False):
    torch, pk, dev = env
    packed = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
    if separate:
        res = []
        for d, p in zip(insts, packed):
            plan = pk.Plan([pk.Instance.from_synth(d, chunk_frames=chunk)], device=dev)
            plan.reset()
            plan.accumulate(p)
            res.append(plan.spectra()[0].cpu().numpy())
        return res
    plan = pk.Plan([pk.Instance.from_synth(d, chunk_frames=chunk) for d in insts], device=dev)
    plan.reset()
    plan.accumulate(packed)
    return [plan.spectra(i)[0].cpu().numpy() for i in range(len(insts))]


@pytest.mark.parametrize("chunk", [0, 4, 2])
def test_grouped_equals_separate(env, chunk):
    say(f"grouped vs separate plans, chunk_frames={chunk}")
    insts = mixed_set()
    a = run(env, insts, chunk)
    b = run(env, insts, chunk, separate=True)
    for i, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), f"instance {i}"


def test_grouped_sub_batches_share_the_inter_pass_buffer(env):
    """One member whose inter-pass data alone exceeds a 128 MiB grouped sub-batch (2^16 points x 300
    frames = 157 MiB), three of one shape class that share a sub-batch (2^14 x 100 frames, 13 MiB each),
    and a 2^18 instance: every sub-batch takes consecutive regions of the plan's one inter-pass buffer;
    spectra bitwise equal to separate plans, and to a second integration of the same plan."""
    torch, pk, dev = env
    insts = [synth.make_correlated_noise(2, 0.3, 1 << 16, 300, seed_extra=900),
             synth.make_correlated_noise(8, 0.2, 1 << 14, 100, seed_extra=901),
             synth.make_correlated_noise(8, 0.4, 1 << 14, 100, seed_extra=902),
             synth.make_correlated_noise(8, 0.1, 1 << 14, 100, seed_extra=903),
             synth.make_correlated_noise(4, 0.3, 1 << 18, 12, seed_extra=904)]
    say("grouped sub-batches in the shared inter-pass buffer")
    a = run(env, insts)
    b = run(env, insts, separate=True)
    for i, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), f"instance {i}"
    c = run(env, insts)
    for i, (x, y) in enumerate(zip(a, c)):
        assert np.array_equal(x, y), f"instance {i} (second plan)"
    # the same plan object again: reset, then every instance's samples in two calls (whole frames each)
    plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev)
    packed = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
    plan.reset()
    plan.accumulate(packed)
    plan.reset()
    cut = [(d["n_frames"] // 2) * d["fft_len"] * d["n_streams"] * d["bits"] // 8 for d in insts]
    plan.accumulate([p[:k] for p, k in zip(packed, cut)])
    plan.accumulate([p[k:] for p, k in zip(packed, cut)])
    for i in range(len(insts)):
        assert np.array_equal(plan.spectra(i)[0].cpu().numpy(), a[i]), f"instance {i} (same plan, two calls)"
    acc, nf, _, _ = oracle.run_instance(insts[1])
    assert np.max(np.abs(a[1] - acc) / np.mean(acc[:, 0:1, :], axis=2, keepdims=True)) < 1e-5


def test_grouped_long_transforms(env):
    """The grouped 1024- and 2048-point pass kernels (2^19 as 1024 x 512, 2^20 as 512 x 2048) in one plan with
    a 2^17 instance, 2- and 8-bit, at least 32 frames each: bitwise equal to separate plans, and every instance's
    Stokes products within 1e-5 of the FP64 oracle (per channel, relative to I)."""
    torch, pk, dev = env
    say("grouped plan of 2^17, 2^19 and 2^20 instances")
    spec = [(17, 8, 40), (19, 2, 32), (19, 8, 34), (20, 8, 32), (20, 2, 33)]
    insts = [synth.make_correlated_noise(bits, 0.1 + 0.08 * i, 1 << e, F, cfg=4, seed_extra=950 + i)
             for i, (e, bits, F) in enumerate(spec)]
    packed = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
    plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev)
    plan.profile_enable(True)
    plan.reset()
    plan.accumulate(packed)
    outs = plan.stokes_all(cals=[(None, None, None, 0.2 * i) for i in range(len(insts))])
    prof = plan.profile_read()
    plan.profile_enable(False)
    torch.cuda.synchronize(dev)
    # one grouped column pass and one row pass per shape class (2^17; 2^19 2-bit and 8-bit; 2^20 2- and 8-bit)
    say(f"  launches {prof}")
    assert prof["colpass"][1] == 5 and prof["rowpass"][1] == 5
    sep = run(env, insts, separate=True)
    for i, d in enumerate(insts):
        assert np.array_equal(plan.spectra(i)[0].cpu().numpy(), sep[i]), f"instance {i}"
        acc, nf, s2, _ = oracle.run_instance(d)
        ref = oracle.stokes(acc, nf, s2, psi=0.2 * i)
        got = outs[i].cpu().numpy().astype(np.float64)
        e = np.max(np.abs(got - ref) / ref[:, 0:1, :], axis=2)
        say(f"  N=2^{spec[i][0]} bits={spec[i][1]} F={spec[i][2]} stokes err {e.ravel().tolist()}")
        assert np.all(e < 1e-5), (i, e)


def test_rebind_uploads_descriptors_again(env):
    """ps_bind onto a fresh (zeroed) workspace, at the same address when the allocator hands it back: the
    grouped launches' descriptors must be uploaded again, and the results equal the first binding's."""
    import ctypes as C
    torch, pk, dev = env
    say("re-bound grouped plan")
    insts = mixed_set()[:5]
    packed = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
    plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev)
    plan.reset()
    plan.accumulate(packed)
    first = [o.clone() for o in plan.stokes_all()]
    torch.cuda.synchronize(dev)
    addr = plan.workspace.data_ptr()
    n = plan.workspace_bytes
    del plan.workspace
    plan._ws_raw = None
    torch.cuda.synchronize(dev)
    raw = torch.zeros(n + 256, dtype=torch.uint8, device=dev)
    off = (-raw.data_ptr()) % 256
    ws = raw[off:off + n]
    say(f"  same address: {ws.data_ptr() == addr}")
    st = pk.lib().ps_bind(plan._h, C.c_void_p(ws.data_ptr()), n, C.c_void_p(plan.stream.cuda_stream))
    assert st == 0, pk.lib().ps_last_error()
    plan._ws_raw, plan.workspace = raw, ws
    plan.reset()
    plan.accumulate(packed)
    again = plan.stokes_all()
    torch.cuda.synchronize(dev)
    for i, (x, y) in enumerate(zip(first, again)):
        assert torch.equal(x, y), f"instance {i}"


def test_grouped_against_oracle(env):
    torch, pk, dev = env
    say("grouped plan vs oracle")
    insts = mixed_set()
    plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev)
    plan.reset()
    plan.accumulate([torch.from_numpy(d["packed"]).to(dev) for d in insts])
    outs = plan.stokes_all()
    torch.cuda.synchronize(dev)
    for i in (1, 4, 10, 12):
        d = insts[i]
        acc, nf, s2, _ = oracle.run_instance(d)
        ref = oracle.stokes(acc, nf, s2)
        got = outs[i].cpu().numpy().astype(np.float64)
        if d["n_frames"] >= 9:
            e = np.max(np.abs(got - ref) / ref[:, 0:1, :])
        else:  # short integrations: normwise
            e = np.max(np.abs(got - ref)) / np.mean(ref[:, 0, :])
        say(f"  instance {i}: N={d['fft_len']} F={d['n_frames']} bits={d['bits']} err {e:.2e}")
        assert e < 1e-5


def test_stokes_all_equals_stokes(env):
    torch, pk, dev = env
    say("stokes_all vs stokes")
    insts = mixed_set()
    plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev)
    plan.reset()
    plan.accumulate([torch.from_numpy(d["packed"]).to(dev) for d in insts])
    rng = np.random.default_rng(3)
    cals = []
    for d in insts:
        P, C = len(d["pairs"]), d["fft_len"] // 2
        g = (1 + 0.05 * (rng.standard_normal((P, C)) + 1j * rng.standard_normal((P, C)))).astype(np.complex64)
        cals.append((torch.from_numpy(g).to(dev), None, None, 0.3))
    outs = plan.stokes_all(cals=cals)
    for i in range(len(insts)):
        one = plan.stokes(i, gain_x=cals[i][0], psi=0.3)
        assert torch.equal(one, outs[i]), f"instance {i}"


def test_graph_replay(env):
    torch, pk, dev = env
    say("graph capture and replay")
    insts = mixed_set()[:12]
    side = torch.cuda.Stream(dev)
    with torch.cuda.stream(side):
        plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev, stream=side)
        packed = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
        outs = [torch.zeros((len(d["pairs"]), 4, d["fft_len"] // 2), dtype=torch.float32, device=dev) for d in insts]
    side.synchronize()

    def integration():
        plan.reset()
        plan.accumulate(packed)
        plan.stokes_all(outs)

    with torch.cuda.stream(side):
        integration()
    side.synchronize()
    eager = [o.clone() for o in outs]
    plan.graph_capture(integration)
    for rep in range(4):
        for o in outs:
            o.zero_()
        side.synchronize()
        plan.graph_replay()
        side.synchronize()
        for i, (o, e) in enumerate(zip(outs, eager)):
            assert torch.equal(o, e), f"replay {rep} instance {i}"
        # eager work between replays, on the same plan
        with torch.cuda.stream(side):
            integration()
        side.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e)
    # the host state after a replay matches the captured integration
    spec, nf = plan.spectra(3)
    assert nf == insts[3]["n_frames"]


def test_graph_errors(env):
    torch, pk, dev = env
    say("graph errors")
    insts = mixed_set()[5:8]  # four-step instances (2^13 .. 2^15): grouped launches with descriptors
    side = torch.cuda.Stream(dev)
    plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev, stream=side)
    with pytest.raises(pk.PolarisError) as e:
        plan.graph_replay()
    assert e.value.code == "PS_ERR_STATE"
    packed = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
    other = [p.clone() for p in packed]
    calls = {"n": 0}

    def changing():
        plan.reset()
        plan.accumulate(packed if calls["n"] == 0 else other)  # new buffers inside the capture
        calls["n"] += 1

    with pytest.raises(pk.PolarisError) as e:
        plan.graph_capture(changing)
    assert e.value.code == "PS_ERR_STATE"
    side.synchronize()
    with pytest.raises(pk.PolarisError) as e:  # nothing was kept
        plan.graph_replay()
    assert e.value.code == "PS_ERR_STATE"
    # the plan still works eagerly
    with torch.cuda.stream(side):
        plan.reset()
        plan.accumulate(other)
    side.synchronize()
    assert plan.spectra(0)[1] == insts[0]["n_frames"]
