"""Oracle gradient (differentiation form) against central finite differences of the oracle's forward.

The leakage model and the tap parameterisation are readings, not the paper's; their gradient is pinned by
finite differences of the pinned forward only.
"""
import numpy as np
import pytest

import oracle
import synth

N, F = 256, 6
NT = 64


@pytest.fixture(scope="module")
def setup():
    rng = np.random.default_rng(11)
    inst = synth.make_correlated_noise(8, 0.25, N, F, seed_extra=9)
    C = N // 2
    taps = 1 + 0.1 * rng.standard_normal(NT)
    gx = 1 + 0.05 * (rng.standard_normal(C) + 1j * rng.standard_normal(C))
    gy = 1 + 0.05 * (rng.standard_normal(C) + 1j * rng.standard_normal(C))
    dt = np.array([[0.02 * np.exp(0.4j), 0.015 * np.exp(2.5j)]])
    weights = rng.standard_normal((1, 4, C))
    return dict(inst=inst, taps=taps, gx=gx[None], gy=gy[None], dt=dt, wts=weights, psi=0.21)


def _loss(s, taps=None, gx=None, gy=None, dt=None):
    taps = s["taps"] if taps is None else taps
    gx = s["gx"] if gx is None else gx
    gy = s["gy"] if gy is None else gy
    dt = s["dt"] if dt is None else dt
    inst = s["inst"]
    w, s2 = oracle.window("taps", N, taps=taps)
    acc, nf = oracle.accumulate(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"], hop=s.get("hop", 0))
    st = oracle.stokes(acc, nf, s2, gain_x=gx, gain_y=gy, dterms=dt, psi=s["psi"])
    # L = sum c * P + 0.5 sum P^2 / scale  (upstream gradient c + P / scale)
    return float(np.sum(s["wts"] * st) + 0.5 * np.sum(st ** 2) / 1e4), st


def _analytic(s):
    inst = s["inst"]
    w, s2 = oracle.window("taps", N, taps=s["taps"])
    acc, nf = oracle.accumulate(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"], hop=s.get("hop", 0))
    _, st = _loss(s)
    g = s["wts"] + st / 1e4
    return oracle.calibrate_backward(inst["packed"], 8, 2, inst["n_samples"], N, w, inst["pairs"], acc, nf, s2, g,
                                     gain_x=s["gx"], gain_y=s["gy"], dterms=s["dt"], psi=s["psi"], taps=s["taps"],
                                     hop=s.get("hop", 0))


def _cfd(f, h):
    return (f(h) - f(-h)) / (2 * h)


def test_gain_gradient(setup):
    s = setup
    g = _analytic(s)
    for k in [0, 1, 17, 100]:
        for part, unit in (("re", 1.0), ("im", 1j)):
            for which in ("gx", "gy"):
                def f(h):
                    arr = s[which].copy()
                    arr[0, k] += unit * h
                    return _loss(s, **{which: arr})[0]
                fd = _cfd(f, 1e-6)
                an = g["d_gain_x" if which == "gx" else "d_gain_y"][0, k]
                an = an.real if part == "re" else an.imag
                assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (which, k, part, fd, an)


def test_dterm_gradient(setup):
    s = setup
    g = _analytic(s)
    for i in range(2):
        for part, unit in (("re", 1.0), ("im", 1j)):
            def f(h):
                arr = s["dt"].copy()
                arr[0, i] += unit * h
                return _loss(s, dt=arr)[0]
            fd = _cfd(f, 1e-6)
            an = g["d_dterms"][0, i]
            an = an.real if part == "re" else an.imag
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (i, part, fd, an)


def test_tap_gradient(setup):
    s = setup
    g = _analytic(s)
    for j in [0, 1, 31, 62, 63]:
        def f(h):
            t = s["taps"].copy()
            t[j] += h
            return _loss(s, taps=t)[0]
        fd = _cfd(f, 1e-5)
        an = g["d_taps"][j]
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (j, fd, an)


@pytest.mark.parametrize("hop", [N // 2, N // 4])
def test_tap_gradient_overlapped_frames(setup, hop):
    """Overlapped segmentation (frame f at sample f * hop): every sample enters several frames, each with its
    own window position."""
    s = dict(setup, hop=hop)
    g = _analytic(s)
    for j in [0, 20, 63]:
        def f(h):
            t = s["taps"].copy()
            t[j] += h
            return _loss(s, taps=t)[0]
        fd = _cfd(f, 1e-5)
        an = g["d_taps"][j]
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (hop, j, fd, an)
