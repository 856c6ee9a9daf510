"""FP64 reference of the post-integration reductions -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this module.  Plain numpy in
FP64, every step written out in the order the paper describes it:

* channel averaging with flagged channels excluded (Sec. 4, sky tests: spectra averaged to coarser channels
  after one spurious channel was flagged);
* the smoothed bandpass H: a least-squares cubic spline with uniform knots every K channels, fitted to a
  long-integration spectrum without the band edges (Sec. 3.3.2: K = 128, 6 % edges);
* the bandpass variation H^_k = H_k / (G_k H) of a series of integrations (Sec. 3.3.2);
* mean and standard deviation of a spectrum, sigma = sqrt(<H^2> - <H>^2) (Sec. 3.3.3);
* the Allan variance of a second difference, Eq. 3 (time lag, TAV, Sec. 3.3.1) and Eq. 4 (frequency
  separation, SAV, Sec. 3.3.3).

Non-finite values (channels outside the fitted band) count as flagged everywhere.
"""
from __future__ import annotations

import numpy as np


def channel_average(x, factor: int, flags=None):
    """x [n_spec][n_chan] -> (mean over each bin's unflagged finite channels [n_spec][n_chan/factor] (NaN when
    none), counts [n_spec][n_chan/factor])."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[None]
    n_spec, n_chan = x.shape
    if factor < 1 or n_chan % factor:
        raise ValueError("factor must divide the channel count")
    use = np.isfinite(x)
    if flags is not None:
        use &= ~np.asarray(flags, dtype=bool)[None, :]
    nb = n_chan // factor
    out = np.full((n_spec, nb), np.nan)
    cnt = np.zeros((n_spec, nb), dtype=np.int64)
    for s in range(n_spec):
        for b in range(nb):
            seg = x[s, b * factor:(b + 1) * factor]
            ok = use[s, b * factor:(b + 1) * factor]
            n = int(ok.sum())
            cnt[s, b] = n
            if n:
                out[s, b] = seg[ok].sum() / n
    return out, cnt


def fit_range(n_chan: int, edge_frac: float):
    """Channels [c0, c1) of the fit: edge_frac of the band dropped at each end."""
    c0 = int(np.floor(edge_frac * n_chan))
    return c0, n_chan - c0


def cubic_bspline_basis(u):
    """The four uniform cubic B-spline pieces at local position u in [0, 1) of an interval."""
    u = np.asarray(u, dtype=np.float64)
    return np.stack([(1 - u) ** 3 / 6, (3 * u ** 3 - 6 * u ** 2 + 4) / 6, (-3 * u ** 3 + 3 * u ** 2 + 3 * u + 1) / 6,
                     u ** 3 / 6], axis=-1)


def bandpass_fit(h, knot_spacing: int = 128, edge_frac: float = 0.06):
    """Smoothed bandpass: the least-squares cubic spline with knots every knot_spacing channels from c0 (one
    coefficient per basis function, n_int + 3 of them), fitted to h[c0:c1]; NaN outside [c0, c1).  Returns
    (smooth [n_chan], coefficients)."""
    h = np.asarray(h, dtype=np.float64)
    n = h.size
    c0, c1 = fit_range(n, edge_frac)
    K = knot_spacing
    n_int = -(-(c1 - c0) // K)
    nb = n_int + 3
    c = np.arange(c0, c1)
    s = (c - c0) / K
    j = np.floor(s).astype(np.int64)
    B = cubic_bspline_basis(s - j)            # [points][4], basis j + q for q = 0..3
    # normal equations A a = r, A banded (each point touches four consecutive basis functions)
    A = np.zeros((nb, nb))
    r = np.zeros(nb)
    for q in range(4):
        np.add.at(r, j + q, B[:, q] * h[c0:c1])
        for p in range(4):
            np.add.at(A, (j + q, j + p), B[:, q] * B[:, p])
    coef = np.linalg.solve(A, r)
    out = np.full(n, np.nan)
    out[c0:c1] = np.sum(B * coef[j[:, None] + np.arange(4)[None, :]], axis=1)
    return out, coef


def bandpass_correct(hk, smooth, gain=None):
    """H^_k = H_k / (G_k H) per spectrum k."""
    hk = np.atleast_2d(np.asarray(hk, dtype=np.float64))
    g = np.ones(hk.shape[0]) if gain is None else np.asarray(gain, dtype=np.float64)
    return hk / (g[:, None] * np.asarray(smooth, dtype=np.float64)[None, :])


def band_stats(x):
    """[n_spec][2]: mean and standard deviation sqrt(<x^2> - <x>^2) over each spectrum's finite channels."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    out = np.full((x.shape[0], 2), np.nan)
    for s in range(x.shape[0]):
        v = x[s][np.isfinite(x[s])]
        if v.size:
            m = v.sum() / v.size
            out[s] = (m, np.sqrt(np.sum((v - m) ** 2) / v.size))
    return out


def allan(x, lags, spacing: float = 1.0, normalize: bool = False):
    """Eq. 3 / Eq. 4 for each row of x [n_series][n_points]: sigma^2(L) = <(x[t+L] - 2 x[t] + x[t-L])^2> /
    (2 (L spacing)^2), the mean over every t with all three samples finite (NaN when none); normalize divides
    the series by the mean of its finite samples first."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    out = np.full((x.shape[0], len(lags)), np.nan)
    for s in range(x.shape[0]):
        v = x[s]
        if normalize:
            v = v / v[np.isfinite(v)].mean()
        for i, L in enumerate(lags):
            if L < 1 or 2 * L >= v.size:
                continue
            d = v[2 * L:] - 2 * v[L:-L] + v[:-2 * L]
            d = d[np.isfinite(d)]
            if d.size:
                out[s, i] = np.sum(d * d) / d.size / (2.0 * (L * spacing) ** 2)
    return out
