"""Oracle pins for the cross-power products and their accumulation (Table 1 products; Sec. 2)."""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def paper_value(name):
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith(name + " "):
                return float(line.split()[1])
    raise KeyError(name)


@pytest.mark.parametrize("bits", [2, 4, 8])
def test_identical_streams_give_xy_equal_xx_exactly(bits):
    inst = synth.make_identical_streams(bits, 512, 6)
    acc, nf, s2, _ = oracle.run_instance(inst)
    assert nf == 6
    assert np.array_equal(acc[0, 2], acc[0, 0])   # Re XY* == XX*
    assert np.all(acc[0, 3] == 0.0)                 # Im XY* == 0
    assert np.array_equal(acc[0, 1], acc[0, 0])


def test_fully_polarized_signal_satisfies_i2_eq_q2_u2_v2():
    inst = synth.make_fully_polarized_f32(1024, 5)
    acc, nf, s2, _ = oracle.run_instance(inst)
    st = oracle.stokes(acc, nf, s2, psi=0.37)
    I, Q, U, V = st[0]
    k = slice(1, None)  # DC was synthesised as zero
    lhs = I[k] ** 2
    rhs = Q[k] ** 2 + U[k] ** 2 + V[k] ** 2
    assert np.max(np.abs(lhs - rhs) / lhs) < 1e-6  # float32 input rounding only
    # and the polarisation state is alpha's: XY*/XX* = conj(alpha)
    alpha = inst["alpha"]
    ratio = (acc[0, 2, k] + 1j * acc[0, 3, k]) / acc[0, 0, k]
    assert np.max(np.abs(ratio - np.conj(alpha))) < 1e-5


def test_correlated_float_noise_recovers_rho():
    rho = 0.3
    inst = synth.make_correlated_noise(32, rho, 1024, 64)
    acc, nf, s2, _ = oracle.run_instance(inst)
    k = slice(1, None)
    r = np.sum(acc[0, 2, k]) / math.sqrt(np.sum(acc[0, 0, k]) * np.sum(acc[0, 1, k]))
    assert abs(r - rho) < 0.02
    assert abs(np.mean(acc[0, 3, k]) / np.mean(acc[0, 0, k])) < 0.02  # no quadrature correlation


def _two_bit_rho(rho):
    """E[q(x) q(y)] / E[q^2] for the 4-level quantiser (thresholds -1, 0, 1; levels -3, -1, 1, 3)."""
    edges = [-np.inf, -1.0, 0.0, 1.0, np.inf]
    lev = [-3.0, -1.0, 1.0, 3.0]
    mvn = stats.multivariate_normal(mean=[0, 0], cov=[[1, rho], [rho, 1]])
    big = 40.0

    def cdf(a, b):
        return mvn.cdf([min(a, big), min(b, big)]) if a > -big and b > -big else 0.0

    e = 0.0
    for i in range(4):
        for j in range(4):
            a0, a1 = max(edges[i], -big), min(edges[i + 1], big)
            b0, b1 = max(edges[j], -big), min(edges[j + 1], big)
            p = cdf(a1, b1) - cdf(a0, b1) - cdf(a1, b0) + cdf(a0, b0)
            e += lev[i] * lev[j] * p
    p_out = 2 * stats.norm.sf(1.0)
    eq2 = 1.0 * (1 - p_out) + 9.0 * p_out
    return e / eq2, eq2


def test_two_bit_quantised_correlation():
    rho = 0.3
    rq, eq2 = _two_bit_rho(rho)
    assert abs(eq2 - 3.538484) < 1e-5
    assert abs(rq - 0.265157) < 2e-5
    inst = synth.make_correlated_noise(2, rho, 1024, 256)
    acc, nf, s2, _ = oracle.run_instance(inst)
    k = slice(1, None)
    r = np.sum(acc[0, 2, k]) / math.sqrt(np.sum(acc[0, 0, k]) * np.sum(acc[0, 1, k]))
    assert abs(r - rq) < 0.012
    # the mean power per channel is E[q^2] per sample: E|X_k|^2 = N E[q^2]
    assert abs(np.mean(acc[0, 0, k]) / (nf * 1024) - eq2) / eq2 < 0.02


def test_radiometer_law():
    """Sec. 3.4: per-channel relative SD of an integrated noise spectrum is 1/sqrt(dnu T) (1/sqrt(F) here)."""
    F = 61
    inst = synth.make_correlated_noise(32, 0.0, 4096, F, seed_extra=3)
    acc, nf, s2, _ = oracle.run_instance(inst)
    xx = acc[0, 0, 1:]
    rel_sd = np.std(xx) / np.mean(xx)
    assert abs(rel_sd - 1 / math.sqrt(F)) / (1 / math.sqrt(F)) < 0.06
    spacing = 16e6 / 2 ** 18
    assert abs(1 / math.sqrt(spacing * 1.0) - paper_value("radiometer_sigma_1s")) < 5e-4


def test_accumulation_independent_of_thread_count():
    inst = synth.make_tiny(n_frames=20)
    w, s2 = oracle.window("hann", 1024)
    args = (inst["packed"], 2, 2, inst["n_samples"], 1024, w, inst["pairs"])
    a1, _ = oracle.accumulate(*args, nthreads=1)
    a4, _ = oracle.accumulate(*args, nthreads=4)
    assert np.array_equal(a1, a4)


def test_accumulation_is_linear_in_frames():
    """Integrating frames [0, F) equals integrating [0, F1) plus [F1, F) (exact for integer-valued sums)."""
    N, F, F1 = 256, 10, 4
    inst = synth.make_correlated_noise(2, 0.2, N, F)
    w, _ = oracle.window("rect", N)
    bpf = N * 2 * 2 // 8  # bytes per frame, 2 streams x 2 bits
    full, _ = oracle.accumulate(inst["packed"], 2, 2, N * F, N, w, [(0, 1)])
    a, _ = oracle.accumulate(inst["packed"][: F1 * bpf], 2, 2, N * F1, N, w, [(0, 1)])
    b, _ = oracle.accumulate(inst["packed"][F1 * bpf:], 2, 2, N * (F - F1), N, w, [(0, 1)])
    assert np.max(np.abs(full - (a + b))) <= 1e-9 * np.max(np.abs(full))


def test_tiny_case_tone_lands_in_channel_100():
    inst = synth.make_tiny()
    acc, nf, s2, _ = oracle.run_instance(inst)
    xx = acc[0, 0]
    assert nf == 64
    assert np.argmax(xx[2:]) + 2 == 100
