"""GPU checks of ps_accumulate_stokes (Sec. 2 functions 2-4 followed by Eq. 2 in one call).

An instance with one accumulator slot gets its Stokes spectra from the epilogue of its last row pass, which
applies the same FP64 arithmetic to the same final sums as the output kernel, so the results must be bitwise
equal to ps_accumulate followed by ps_stokes (and the accumulators, read back as spectra, too).  Instances
that cannot take the fused epilogue go through one grouped output launch; same bitwise bar.  Against the
FP64 oracle the bar is the FP32 path's: max_k |P_gpu - P_ref| / I_ref,k <= 1e-5 per Stokes product.
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
def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def pk():
    import paper_1412_1256_amd as pk
    pk.lib()
    return pk


def _cal_tensors(torch, dev, C_, P, seed):
    rng = np.random.default_rng(seed)
    g = 1 + 0.08 * (rng.standard_normal((2, P, C_)) + 1j * rng.standard_normal((2, P, C_)))
    gx = torch.from_numpy(np.stack([g[0].real, g[0].imag], -1).astype(np.float32)).to(dev)
    gy = torch.from_numpy(np.stack([g[1].real, g[1].imag], -1).astype(np.float32)).to(dev)
    d = 0.02 * np.exp(1j * rng.uniform(0, 2 * np.pi, (P, 2)))
    dt = torch.from_numpy(np.stack([d[:, 0].real, d[:, 0].imag, d[:, 1].real, d[:, 1].imag], -1)
                          .astype(np.float32)).to(dev)
    return gx, gy, dt


CASES = {
    # name: (instance maker, Instance overrides, schedule (None = default), calibrated, feed, expect fused)
    "paper_2e18_one_slot": (lambda: synth.make_paper(n_frames=61), {}, dict(rowpass_slots=1), True, "linear", True),
    "paper_2e18_default": (lambda: synth.make_paper(n_frames=61), {}, None, True, "linear", None),
    "2e16_int8_circular": (lambda: synth.make_correlated_noise(8, 0.2, 1 << 16, 40, seed_extra=61), {},
                           dict(rowpass_slots=1), True, "circular", True),
    "2e14_2bit_hann_overlap": (lambda: synth.make_correlated_noise(2, 0.3, 1 << 14, 48, seed_extra=62),
                               dict(window="hann", hop=1 << 13), dict(rowpass_slots=1), False, "linear", True),
    "2e12_single_pass": (lambda: synth.make_correlated_noise(2, 0.3, 1 << 12, 64, seed_extra=63), {}, None,
                         True, "linear", False),
    "2e15_int8_many_slots": (lambda: synth.make_correlated_noise(8, 0.1, 1 << 15, 70, seed_extra=64), {}, None,
                             False, "linear", False),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fused_equals_accumulate_then_stokes(pk, torch_dev, name):
    torch, dev = torch_dev
    make, over, sched, calibrated, feed, expect_fused = CASES[name]
    say(f"accumulate_stokes vs accumulate + stokes: {name}")
    inst = make()
    I = pk.Instance.from_synth(inst, **over)
    S = None if sched is None else [pk.Schedule(**sched)]
    packed = torch.from_numpy(inst["packed"]).to(dev)
    cal = {}
    if calibrated:
        gx, gy, dt = _cal_tensors(torch, dev, I.channels, I.n_pairs, 7)
        cal = dict(gain_x=gx, gain_y=gy, dterms=dt)
    a = pk.Plan([I], device=dev, schedules=S)
    b = pk.Plan([I], device=dev, schedules=S)
    a.profile_enable(True)
    a.reset()
    fused = a.accumulate_stokes(packed, psi=0.4, feed=feed, **cal)[0]
    prof = a.profile_read()
    a.profile_enable(False)
    b.reset()
    b.accumulate(packed)
    sep = b.stokes(psi=0.4, feed=feed, **cal)
    sa, na = a.spectra()
    sb, nb = b.spectra()
    torch.cuda.synchronize(dev)
    assert na == nb
    say(f"  kernels {sorted(prof)}")
    if expect_fused is not None:
        assert ("stokes" not in prof) == expect_fused, prof
    assert torch.equal(fused, sep), (fused - sep).abs().max().item()
    assert torch.equal(sa, sb)


def test_fused_split_calls(pk, torch_dev):
    """accumulate(first part) then accumulate_stokes(rest) equals the whole integration in one call."""
    torch, dev = torch_dev
    say("split: accumulate + accumulate_stokes")
    inst = synth.make_correlated_noise(8, 0.25, 1 << 16, 50, seed_extra=65)
    I = pk.Instance.from_synth(inst)
    S = [pk.Schedule(rowpass_slots=1)]
    packed = torch.from_numpy(inst["packed"]).to(dev)
    cut = (17 << 16) * 2  # 17 frames of two int8 streams
    a = pk.Plan([I], device=dev, schedules=S)
    a.reset()
    a.accumulate(packed[:cut])
    got = a.accumulate_stokes(packed[cut:], psi=-0.3)[0]
    b = pk.Plan([I], device=dev, schedules=S)
    b.reset()
    b.accumulate(packed)
    ref = b.stokes(psi=-0.3)
    torch.cuda.synchronize(dev)
    assert torch.equal(got, ref)


def test_fused_paper_config_vs_oracle(pk, torch_dev):
    """The paper-shaped integration (2 int8 streams, 2^18 points, 61 frames) through the fused epilogue."""
    torch, dev = torch_dev
    say("fused paper config vs oracle")
    inst = synth.make_paper()
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2, psi=0.25)
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev, schedules=[pk.Schedule(rowpass_slots=1)])
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.reset()
    got = plan.accumulate_stokes(packed, psi=0.25)[0]
    torch.cuda.synchronize(dev)
    got = got.cpu().numpy().astype(np.float64)
    e = np.max(np.abs(got - ref) / ref[:, 0:1, :], axis=2)
    say(f"  stokes err {e.tolist()}")
    assert np.all(e < TOL), e


def test_fused_multi_instance_plan(pk, torch_dev):
    """A grouped plan: Stokes from one grouped output launch after the accumulation, same as stokes_all."""
    torch, dev = torch_dev
    say("accumulate_stokes on a two-instance plan")
    i1 = synth.make_correlated_noise(8, 0.2, 1 << 14, 40, seed_extra=66)
    i2 = synth.make_correlated_noise(2, 0.4, 1 << 16, 20, seed_extra=67)
    insts = [pk.Instance.from_synth(i1), pk.Instance.from_synth(i2)]
    packed = [torch.from_numpy(i["packed"]).to(dev) for i in (i1, i2)]
    a = pk.Plan(insts, device=dev)
    a.reset()
    got = a.accumulate_stokes(packed, cals=[(None, None, None, 0.1), (None, None, None, -0.2)])
    b = pk.Plan(insts, device=dev)
    b.reset()
    b.accumulate(packed)
    ref = b.stokes_all(cals=[(None, None, None, 0.1), (None, None, None, -0.2)])
    torch.cuda.synchronize(dev)
    for g, r in zip(got, ref):
        assert torch.equal(g, r)


def test_fused_no_frames_is_an_error(pk, torch_dev):
    torch, dev = torch_dev
    plan = pk.Plan([pk.Instance(fft_len=1 << 14, bits=8)], device=dev)
    plan.reset()
    empty = torch.empty(0, dtype=torch.uint8, device=dev)
    with pytest.raises(pk.PolarisError) as ei:
        plan.accumulate_stokes(empty)
    assert ei.value.code == "PS_ERR_STATE"
