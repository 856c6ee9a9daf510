"""Oracle pins for calibration and full Stokes (Sec. 2.1, Eq. 2)."""
import numpy as np
import pytest

import oracle


def _random_stokes(rng, C, pol=0.6):
    I = rng.uniform(1.0, 3.0, C)
    Q, U, V = (rng.uniform(-1, 1, (3, C)) * pol * I / np.sqrt(3))
    return I, Q, U, V


def _coherency_to_acc(XX, YY, XY, F, s2):
    acc = np.stack([XX, YY, XY.real, XY.imag])[None] * (F * s2)
    return acc


def test_linear_feed_coherency_is_recovered_at_zero_angle():
    """XX* = I+Q, YY* = I-Q, XY* = U+iV for linear feeds at psi = 0 (textbook relation)."""
    rng = np.random.default_rng(1)
    C, F, s2 = 64, 7, 300.0
    I, Q, U, V = _random_stokes(rng, C)
    acc = _coherency_to_acc(I + Q, I - Q, U + 1j * V, F, s2)
    st = oracle.stokes(acc, F, s2)
    assert np.allclose(st[0], np.stack([I, Q, U, V]), rtol=0, atol=1e-12)


@pytest.mark.parametrize("psi", [0.0, 0.3, -1.2, np.pi / 4])
def test_parallactic_angle_rotates_q_u_by_twice_psi(psi):
    rng = np.random.default_rng(2)
    C, F, s2 = 50, 3, 10.0
    I, Q, U, V = _random_stokes(rng, C)
    acc = _coherency_to_acc(I + Q, I - Q, U + 1j * V, F, s2)
    st = oracle.stokes(acc, F, s2, psi=psi)[0]
    c, s = np.cos(2 * psi), np.sin(2 * psi)
    assert np.allclose(st[0], I, atol=1e-12)
    assert np.allclose(st[1], c * Q - s * U, atol=1e-12)
    assert np.allclose(st[2], s * Q + c * U, atol=1e-12)
    assert np.allclose(st[3], V, atol=1e-12)
    assert np.allclose(st[1] ** 2 + st[2] ** 2, Q ** 2 + U ** 2, atol=1e-11)


def test_gains_and_leakage_are_removed():
    """Observed coherency G J C J^H G^H (forward measurement model) calibrates back to C."""
    rng = np.random.default_rng(3)
    C, F, s2 = 40, 11, 64.0
    I, Q, U, V = _random_stokes(rng, C)
    gx = 1 + 0.2 * (rng.standard_normal(C) + 1j * rng.standard_normal(C))
    gy = 1 + 0.2 * (rng.standard_normal(C) + 1j * rng.standard_normal(C))
    dx, dy = 0.05 * np.exp(0.7j), 0.03 * np.exp(-2.1j)
    Cm = np.zeros((C, 2, 2), dtype=complex)
    Cm[:, 0, 0] = I + Q
    Cm[:, 1, 1] = I - Q
    Cm[:, 0, 1] = U + 1j * V
    Cm[:, 1, 0] = U - 1j * V
    G = np.zeros((C, 2, 2), dtype=complex)
    G[:, 0, 0] = gx
    G[:, 1, 1] = gy
    J = np.array([[1, dx], [dy, 1]])
    E = G @ J
    M = E @ Cm @ np.conj(np.transpose(E, (0, 2, 1)))
    acc = _coherency_to_acc(M[:, 0, 0].real, M[:, 1, 1].real, M[:, 0, 1], F, s2)
    st = oracle.stokes(acc, F, s2, gain_x=gx[None], gain_y=gy[None], dterms=np.array([[dx, dy]]))
    assert np.allclose(st[0], np.stack([I, Q, U, V]), atol=1e-11)
    # without leakage terms the same gains alone divide the products exactly as Eq. 2 prints
    M0 = G @ Cm @ np.conj(np.transpose(G, (0, 2, 1)))
    acc0 = _coherency_to_acc(M0[:, 0, 0].real, M0[:, 1, 1].real, M0[:, 0, 1], F, s2)
    st0 = oracle.stokes(acc0, F, s2, gain_x=gx[None], gain_y=gy[None])
    assert np.allclose(st0[0], np.stack([I, Q, U, V]), atol=1e-11)


def test_unit_gains_zero_leakage_is_identity():
    rng = np.random.default_rng(4)
    C, F, s2 = 30, 2, 5.0
    acc = rng.uniform(0.5, 2, (1, 4, C))
    a = oracle.stokes(acc, F, s2)
    b = oracle.stokes(acc, F, s2, gain_x=np.ones((1, C)), gain_y=np.ones((1, C)), dterms=np.zeros((1, 2)))
    assert np.array_equal(a, b)


def test_unpolarized_noise_has_small_q_u_v():
    import synth
    inst = synth.make_correlated_noise(8, 0.0, 2048, 40)
    acc, nf, s2, _ = oracle.run_instance(inst)
    st = oracle.stokes(acc, nf, s2)[0]
    I = st[0][1:]
    for q in st[1:]:
        assert np.sqrt(np.mean((q[1:] / I) ** 2)) < 3 / np.sqrt(nf)


# ------------------------------------------------------------------------------------------------
# circular feeds (a reading: R = (X + iY)/sqrt 2, L = (X - iY)/sqrt 2; the paper gives no formula)

def _coherency_acc(X, Y):
    """raw products acc[1][4][C] (XX*, YY*, Re XY*, Im XY*) of one frame of spectra X, Y"""
    xy = X * np.conj(Y)
    return np.stack([np.abs(X) ** 2, np.abs(Y) ** 2, xy.real, xy.imag])[None]


@pytest.mark.parametrize("psi", [0.0, 0.3, -1.1])
def test_circular_feeds_see_the_same_sky(psi):
    """The same field sampled by linear feeds (X, Y) and by circular feeds (R, L) gives the same Stokes."""
    rng = np.random.default_rng(21)
    C = 64
    X = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    Y = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    R = (X + 1j * Y) / np.sqrt(2.0)
    L = (X - 1j * Y) / np.sqrt(2.0)
    lin = oracle.stokes(_coherency_acc(X, Y), 1, 1.0, psi=psi)
    circ = oracle.stokes(_coherency_acc(R, L), 1, 1.0, psi=psi, feed="circular")
    assert np.allclose(lin, circ, rtol=0, atol=1e-12 * np.max(np.abs(lin)))


def test_circular_pure_states():
    C = 8
    ones = np.ones(C, dtype=complex)
    # right-circular only: V = I; left only: V = -I
    r = oracle.stokes(_coherency_acc(ones, 0 * ones), 1, 1.0, feed="circular")[0]
    assert np.allclose(r[0], 0.5) and np.allclose(r[3], 0.5) and np.allclose(r[1:3], 0.0)
    l_ = oracle.stokes(_coherency_acc(0 * ones, ones), 1, 1.0, feed="circular")[0]
    assert np.allclose(l_[3], -0.5)
    # equal R and L in phase: linear polarization, Q = I, and psi rotates it into U
    q = oracle.stokes(_coherency_acc(ones, ones), 1, 1.0, feed="circular")[0]
    assert np.allclose(q[1], q[0]) and np.allclose(q[2], 0.0) and np.allclose(q[3], 0.0)
    u = oracle.stokes(_coherency_acc(ones, ones), 1, 1.0, psi=np.pi / 4, feed="circular")[0]
    assert np.allclose(u[2], u[0]) and np.allclose(u[1], 0.0, atol=1e-15)
