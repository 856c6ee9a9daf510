"""The allocation-free bandpass fit (ps_bandpass_fit_static) against ps_bandpass_fit, through the C ABI.

Both run the same kernels on the same inputs; the static variant takes its work buffer from the library's
static device array instead of the caller's.  Two calls in a row, the second smaller than the first (the array
keeps the first call's contents), must each equal the caller-buffer call exactly (NaN outside the fitted band
in the same channels); a fit needing more scratch than the array holds is refused before any launch.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1412_1256_amd as pk
    pk.lib()
    return torch, torch.device("cuda:0"), pk


def _bandpass(n_chan, seed):
    rng = np.random.default_rng(seed)
    x = np.linspace(0.0, 1.0, n_chan)
    h = 1.0 + 0.3 * np.sin(7.0 * x) + 0.1 * x * x + 0.01 * rng.standard_normal(n_chan)
    return h.astype(np.float32)


def _same(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


def test_static_fit_matches_caller_buffer_fit(env):
    torch, dev, pk = env
    L = pk.lib()
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    for n_chan, knots, edge, seed in [(131072, 128, 0.06, 1), (32768, 64, 0.06, 2)]:
        print(f"static bandpass fit n_chan={n_chan} knots={knots}", flush=True)
        h = torch.from_numpy(_bandpass(n_chan, seed)).to(dev)
        ref = pk.bandpass_fit(h, knots, edge)
        got = torch.full_like(h, 7.0)
        st = L.ps_bandpass_fit_static(C.c_void_p(h.data_ptr()), n_chan, knots, edge, C.c_void_p(got.data_ptr()),
                                      stream)
        assert st == 0, L.ps_last_error().decode()
        torch.cuda.synchronize(dev)
        assert _same(got, ref)
        assert torch.isfinite(got[n_chan // 2]).item()


def test_static_fit_refuses_more_than_its_scratch(env):
    torch, dev, pk = env
    L = pk.lib()
    n_chan = 131072
    h = torch.from_numpy(_bandpass(n_chan, 3)).to(dev)
    out = torch.full_like(h, 7.0)
    # 64-channel knots: 1806 coefficients, more than the 1024 the static scratch holds
    st = L.ps_bandpass_fit_static(C.c_void_p(h.data_ptr()), n_chan, 64, 0.06, C.c_void_p(out.data_ptr()), None)
    assert pk.STATUS[st] == "PS_ERR_SIZE"
    assert "static buffer" in L.ps_last_error().decode()
    torch.cuda.synchronize(dev)
    assert torch.all(out == 7.0).item()
