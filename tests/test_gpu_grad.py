"""Differentiation form on the GPU against the FP64 oracle's analytic gradient (itself pinned by finite
differences of the pinned forward).

Bounds:
  * gains, per channel: |d_k| <= 1e-5 * s_k with s_k = |g_k|_1 I_k, the size of the terms whose sum is the
    channel's gradient (upstream gradient of the channel's four Stokes products times its total power): a
    channel whose gradient is small because its terms cancel is held to the rounding of those terms, not to
    the largest channel's gradient;
  * leakage terms (sums over all channels): max|d| / max|ref| <= 1e-5;
  * window taps (sums over every sample of FP32 inverse transforms), per tap: |d_j| <= 1e-4 max(|ref_j|,
    1e-2 max|ref|).
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


def _cplx(rng, shape, sd):
    return sd * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def _case(N, F, seed, bits=8, taps=True, n_taps=64):
    rng = np.random.default_rng(seed)
    inst = synth.make_correlated_noise(bits, 0.3, N, F, seed_extra=seed, window="taps" if taps else "rect")
    C = N // 2
    d = dict(inst=inst, C=C,
             gx=(1 + _cplx(rng, (1, C), 0.05)).astype(np.complex64),
             gy=(1 + _cplx(rng, (1, C), 0.05)).astype(np.complex64),
             dt=(0.02 * np.exp(1j * rng.uniform(0, 6.28, (1, 2)))).astype(np.complex64),
             taps=(1 + 0.1 * rng.standard_normal(n_taps)).astype(np.float32),
             g=rng.standard_normal((1, 4, C)).astype(np.float32), psi=0.37)
    return d


def _oracle(d, taps=True):
    inst = d["inst"]
    t = d["taps"].astype(np.float64) if taps else None
    w, s2 = oracle.window("taps" if taps else "rect", inst["fft_len"], taps=t)
    acc, nf = oracle.accumulate(inst["packed"], inst["bits"], 2, inst["n_samples"], inst["fft_len"], w, inst["pairs"])
    st = oracle.stokes(acc, nf, s2, gain_x=d["gx"].astype(np.complex128), gain_y=d["gy"].astype(np.complex128),
                       dterms=d["dt"].astype(np.complex128), psi=d["psi"])
    gr = oracle.calibrate_backward(inst["packed"], inst["bits"], 2, inst["n_samples"], inst["fft_len"], w,
                                   inst["pairs"], acc, nf, s2, d["g"].astype(np.float64),
                                   gain_x=d["gx"].astype(np.complex128), gain_y=d["gy"].astype(np.complex128),
                                   dterms=d["dt"].astype(np.complex128), psi=d["psi"], taps=t)
    return st, gr


def _gpu(env, d, taps=True, want=("gain_x", "gain_y", "dterms", "taps"), split=False):
    """split: the integration in two accumulate calls, so the backward transforms the frames again instead
    of using the forward's inter-pass buffer"""
    torch, pk, dev = env
    inst = d["inst"]
    plan = pk.Plan([pk.Instance.from_synth(inst, n_taps=len(d["taps"]))], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    if taps:
        plan.set_window_taps(torch.from_numpy(d["taps"]).to(dev))
    plan.reset()
    if split:
        N, F, per_t = inst["fft_len"], inst["n_frames"], 2 * inst["bits"] // 8
        cut = (F // 2) * N * per_t
        plan.accumulate(packed[:cut])
        plan.accumulate(packed[cut:])
    else:
        plan.accumulate(packed)
    gx = torch.from_numpy(d["gx"]).to(dev)
    gy = torch.from_numpy(d["gy"]).to(dev)
    dt = torch.from_numpy(d["dt"]).to(dev)
    st = plan.stokes(gain_x=gx, gain_y=gy, dterms=dt, psi=d["psi"])
    g = torch.from_numpy(d["g"]).to(dev)
    out = plan.calibrate_backward(packed, g, gain_x=gx, gain_y=gy, dterms=dt, psi=d["psi"],
                                  want=want if taps else tuple(w for w in want if w != "taps"))
    torch.cuda.synchronize(dev)
    res = {k: v.cpu().numpy() for k, v in out.items()}
    return st.cpu().numpy().astype(np.float64), res


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _per_channel(got, ref, g, I):
    """max_k |got_k - ref_k| / (|g_k|_1 I_k): g [P][4][C] upstream gradient, I [P][C] total power"""
    scale = np.sum(np.abs(g), axis=1) * I
    return float(np.max(np.abs(got - ref) / scale))


def _per_tap(got, ref):
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-2 * np.max(np.abs(ref)))))


# (n_taps 512 at N = 4096: a 256-sample block spans too many taps for the one-pass tap gradient, so the
# two-kernel form runs; split: the column pass is recomputed in the backward)
@pytest.mark.parametrize("N,F,taps,n_taps,split", [(2048, 20, False, 64, False), (4096, 10, True, 64, False),
                                                   (1 << 16, 6, True, 64, False), (4096, 10, True, 512, False),
                                                   (4096, 12, True, 64, True), (2048, 20, False, 64, True)])
def test_gradients_match_oracle(env, N, F, taps, n_taps, split):
    say(f"gradients N={N} F={F} taps={taps} n_taps={n_taps} split={split}")
    d = _case(N, F, seed=N + F, n_taps=n_taps)
    st_ref, gr = _oracle(d, taps)
    st, out = _gpu(env, d, taps, split=split)
    I = st_ref[0, 0]
    e_st = np.max(np.abs(st[0] - st_ref[0]) / I, axis=1)
    gx = out["gain_x"][..., 0] + 1j * out["gain_x"][..., 1]
    gy = out["gain_y"][..., 0] + 1j * out["gain_y"][..., 1]
    dt = out["dterms"][:, 0::2] + 1j * out["dterms"][:, 1::2]
    Ik = st_ref[:, 0, :]
    e = dict(stokes=float(e_st.max()), gx=_per_channel(gx, gr["d_gain_x"], d["g"], Ik),
             gy=_per_channel(gy, gr["d_gain_y"], d["g"], Ik), dt=_rel(dt, gr["d_dterms"]),
             gx_normwise=_rel(gx, gr["d_gain_x"]))
    if taps:
        e["taps"] = _per_tap(out["taps"], gr["d_taps"])
    say(f"  errors {e}")
    assert e["stokes"] < 1e-5
    assert e["gx"] < 1e-5 and e["gy"] < 1e-5 and e["dt"] < 1e-5
    if taps:
        assert e["taps"] < 1e-4


def test_differentiation_config_autograd(env):
    """2 pols, 2^16-pt frames, 128 frames, learnable gains, leakage and 64 taps; MSE loss against the
    calibrator's Stokes; torch.autograd through the adjoint vs the oracle gradient."""
    torch, pk, dev = env
    from paper_1412_1256_amd.autograd import stokes as stokes_fn
    say("differentiation configuration (autograd)")
    inst = synth.make_differentiation()
    N, C = inst["fft_len"], inst["fft_len"] // 2
    gx0 = inst["init_gain_x"].astype(np.complex64)[None]
    gy0 = inst["init_gain_y"].astype(np.complex64)[None]
    taps0 = np.ones(64, dtype=np.float32)
    tgt = inst["target"]
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    gx = torch.from_numpy(gx0).to(dev).requires_grad_()
    gy = torch.from_numpy(gy0).to(dev).requires_grad_()
    dt = torch.zeros((1, 2), dtype=torch.complex64, device=dev).requires_grad_()
    taps = torch.from_numpy(taps0).to(dev).requires_grad_()
    iquv = stokes_fn(plan, packed, gx, gy, dt, taps, psi=0.0)
    upstream = []
    iquv.register_hook(lambda gr_: upstream.append(gr_.detach().clone()))
    T = torch.from_numpy(tgt).to(dev).float()
    loss = torch.mean((iquv - T) ** 2 / T[:, 0:1] ** 2)
    loss.backward()
    torch.cuda.synchronize(dev)
    # oracle: the adjoint at the upstream gradient the node received, dL/dP = 2 (P - T) / (T_I^2 * 4C) of the
    # GPU's own P (the oracle's P differs by the forward's rounding, which near the fit, P ~ T, is a large
    # relative change of P - T and so of the upstream gradient itself)
    w, s2 = oracle.window("taps", N, taps=taps0.astype(np.float64))
    acc, nf = oracle.accumulate(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"])
    st = oracle.stokes(acc, nf, s2, gain_x=gx0.astype(np.complex128), gain_y=gy0.astype(np.complex128),
                       dterms=np.zeros((1, 2)), psi=0.0)
    g = upstream[0].cpu().numpy().astype(np.float64)
    g_own = 2 * (st - tgt) / (tgt[:, 0:1] ** 2) / st.size
    say(f"  upstream gradient: GPU vs oracle-forward max rel {np.max(np.abs(g - g_own)) / np.max(np.abs(g_own)):.2e}")
    gr = oracle.calibrate_backward(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"], acc, nf, s2, g,
                                   gain_x=gx0.astype(np.complex128), gain_y=gy0.astype(np.complex128),
                                   dterms=np.zeros((1, 2)), psi=0.0, taps=taps0.astype(np.float64))
    Ik = st[:, 0, :]
    e = dict(gx=_per_channel(gx.grad.cpu().numpy(), gr["d_gain_x"], g, Ik),
             gy=_per_channel(gy.grad.cpu().numpy(), gr["d_gain_y"], g, Ik),
             dt=_rel(dt.grad.cpu().numpy(), gr["d_dterms"]), taps=_per_tap(taps.grad.cpu().numpy(), gr["d_taps"]))
    say(f"  errors {e}")
    assert e["gx"] < 1e-5 and e["gy"] < 1e-5 and e["dt"] < 1e-5 and e["taps"] < 1e-4


def test_interleaved_forwards_refuse_a_stale_backward(env):
    """Two forwards on one plan, then the first one's backward: the plan now holds the second integration, so
    the first node must refuse rather than return the second's gradients; a backward right after its own
    forward still works."""
    torch, pk, dev = env
    from paper_1412_1256_amd.autograd import stokes as stokes_fn
    say("interleaved forwards")
    d1, d2 = _case(4096, 8, seed=71), _case(4096, 8, seed=72)
    plan = pk.Plan([pk.Instance.from_synth(d1["inst"])], device=dev)
    p1 = torch.from_numpy(d1["inst"]["packed"]).to(dev)
    p2 = torch.from_numpy(d2["inst"]["packed"]).to(dev)
    gx = torch.from_numpy(d1["gx"]).to(dev).requires_grad_()
    taps = torch.from_numpy(d1["taps"]).to(dev).requires_grad_()
    y1 = stokes_fn(plan, p1, gain_x=gx, taps=taps)
    y2 = stokes_fn(plan, p2, gain_x=gx, taps=taps)
    with pytest.raises(pk.PolarisError) as e:
        y1.sum().backward()
    assert e.value.code == "PS_ERR_STATE"
    y2.sum().backward()  # the latest forward's backward is valid
    torch.cuda.synchronize(dev)
    assert torch.isfinite(gx.grad).all().item() and torch.isfinite(taps.grad).all().item()
    # a new forward after set_window_taps alone also invalidates the previous node
    y3 = stokes_fn(plan, p1, gain_x=gx, taps=taps)
    plan.set_window_taps(torch.ones(64, device=dev))
    with pytest.raises(pk.PolarisError):
        y3.sum().backward()


def test_backward_argument_errors(env):
    torch, pk, dev = env
    say("backward errors")
    d = _case(1024, 4, seed=3)
    inst = d["inst"]
    plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    plan.reset()
    plan.accumulate(packed)
    g = torch.zeros((1, 4, 512), dtype=torch.float32, device=dev)
    with pytest.raises(pk.PolarisError) as e:
        plan.calibrate_backward(packed[: packed.numel() // 2], g)
    assert e.value.code == "PS_ERR_STATE"
    rect = pk.Plan([pk.Instance(fft_len=1024, bits=8)], device=dev)
    rect.reset()
    rect.accumulate(packed)
    with pytest.raises(pk.PolarisError) as e:
        rect.set_window_taps(torch.ones(64, device=dev))
    assert e.value.code == "PS_ERR_ARG"
