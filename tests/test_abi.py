"""Host-side checks of the C ABI: exported symbols and argument validation (no GPU work)."""
import ctypes as C
import os
import re

import pytest

import paper_1412_1256_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polaris.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ps_[a-z_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert "ps_plan" in names and "ps_accumulate" in names and "ps_stokes" in names
    assert "ps_calibrate_backward" in names
    L = C.CDLL(pk.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_instance_struct_layout_matches_header():
    assert C.sizeof(pk._Instance) == 88
    assert pk._Instance.fft_len.offset == 64 and pk._Instance.hop.offset == 80
    assert C.sizeof(pk._Cal) == 40 and pk._Cal.feed.offset == 32


def _plan(**kw):
    base = dict(fft_len=1024, bits=2)
    base.update(kw)
    inst = pk.Instance(**base)
    arr = (pk._Instance * 1)(inst.to_c())
    h = C.c_void_p()
    n = C.c_size_t()
    st = pk.lib().ps_plan(arr, 1, C.byref(h), C.byref(n))
    return st, h, n.value


def test_valid_plan_reports_aligned_workspace():
    st, h, n = _plan()
    assert st == 0 and n > 0 and n % 256 == 0
    # accumulators (32 bytes per channel and pair) plus the 64-frame FP32 inter-pass buffer fit inside
    assert n >= 64 * 1024 * 8 + 512 * 32
    assert pk.lib().ps_destroy(h) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(bits=3), "PS_ERR_ARG"),
    (dict(fft_len=1000), "PS_ERR_ARG"),
    (dict(fft_len=64), "PS_ERR_UNSUPPORTED"),
    (dict(fft_len=1 << 23), "PS_ERR_UNSUPPORTED"),
    (dict(pairs=((0, 2),)), "PS_ERR_ARG"),
    (dict(n_streams=0), "PS_ERR_ARG"),
    (dict(window="taps", n_taps=1), "PS_ERR_ARG"),
    (dict(window=7), "PS_ERR_ARG"),
    (dict(chunk_frames=-1), "PS_ERR_ARG"),
    (dict(precision=5), "PS_ERR_ARG"),
    (dict(accum=3), "PS_ERR_ARG"),
    (dict(accum="kahan32"), "PS_ERR_UNSUPPORTED"),
    (dict(fft_len=1 << 20, precision="fp16"), "PS_ERR_UNSUPPORTED"),
    (dict(fft_len=1 << 12, precision="bf16"), "PS_ERR_UNSUPPORTED"),
    (dict(fft_len=1 << 16, precision="fp16", window="taps", n_taps=64), "PS_ERR_UNSUPPORTED"),
    (dict(hop=384), "PS_ERR_ARG"),
    (dict(hop=64), "PS_ERR_ARG"),
    (dict(hop=2048), "PS_ERR_ARG"),
    (dict(hop=-512), "PS_ERR_ARG"),
])
def test_plan_rejects_bad_instances(kw, code):
    st, h, n = _plan(**kw)
    assert pk.STATUS[st] == code, pk.lib().ps_last_error()
    assert not h.value
    assert len(pk.lib().ps_last_error()) > 0


@pytest.mark.parametrize("log2n", [16, 17, 18])
@pytest.mark.parametrize("precision,accum", [("fp16", "kahan32"), ("bf16", "fp64")])
def test_reduced_precision_plans(log2n, precision, accum):
    st, h, n = _plan(fft_len=1 << log2n, precision=precision, accum=accum)
    assert st == 0, pk.lib().ps_last_error()
    assert n % 256 == 0
    assert pk.lib().ps_destroy(h) == 0


def test_calls_before_bind_are_state_errors():
    st, h, n = _plan()
    assert st == 0
    L = pk.lib()
    assert pk.STATUS[L.ps_reset(h)] == "PS_ERR_STATE"
    ptrs = (C.c_void_p * 1)(None)
    ns = (C.c_int64 * 1)(0)
    assert pk.STATUS[L.ps_accumulate(h, ptrs, ns)] == "PS_ERR_STATE"
    assert pk.STATUS[L.ps_stokes(h, 0, None, C.c_void_p(16))] == "PS_ERR_STATE"
    outs = (C.c_void_p * 1)(16)
    assert pk.STATUS[L.ps_accumulate_stokes(h, ptrs, ns, None, outs)] == "PS_ERR_STATE"
    L.ps_destroy(h)


def test_bind_rejects_bad_workspace_before_any_device_call():
    st, h, n = _plan()
    L = pk.lib()
    assert pk.STATUS[L.ps_bind(h, None, n, None)] == "PS_ERR_WORKSPACE"
    assert pk.STATUS[L.ps_bind(h, C.c_void_p(4096 + 8), n, None)] == "PS_ERR_WORKSPACE"
    assert pk.STATUS[L.ps_bind(h, C.c_void_p(4096), n - 256, None)] == "PS_ERR_WORKSPACE"
    L.ps_destroy(h)


def test_status_strings():
    L = pk.lib()
    for code, name in pk.STATUS.items():
        assert L.ps_status_string(code).decode() == name


def test_unpack_argument_errors():
    L = pk.lib()
    assert pk.STATUS[L.ps_unpack(None, 8, 2, 10, C.c_void_p(16), None)] == "PS_ERR_ARG"
    assert pk.STATUS[L.ps_unpack(C.c_void_p(16), 5, 2, 10, C.c_void_p(16), None)] == "PS_ERR_ARG"
    assert pk.STATUS[L.ps_unpack(C.c_void_p(16), 8, 9, 10, C.c_void_p(16), None)] == "PS_ERR_ARG"
    assert L.ps_unpack(C.c_void_p(16), 8, 2, 0, C.c_void_p(16), None) == 0  # empty: nothing enqueued


def test_schedule_candidates_and_scheduled_plans():
    inst = pk.Instance(fft_len=1 << 18, bits=8)
    cands = pk.schedule_candidates(inst)
    splits = {c.log2_n1 for c in cands}
    assert splits == {8, 9, 10}
    assert pk.Schedule(9, 16, 8, 1, 1) in cands and pk.Schedule(9, 8, 4, 2, 2) in cands
    for c in cands:
        arr = (pk._Instance * 1)(inst.to_c())
        sarr = (pk._Schedule * 1)(c.to_c())
        h = C.c_void_p()
        n = C.c_size_t()
        assert pk.lib().ps_plan_scheduled(arr, sarr, 1, C.byref(h), C.byref(n)) == 0
        pk.lib().ps_destroy(h)
    # 16-bit passes: default schedule only
    assert pk.schedule_candidates(pk.Instance(fft_len=1 << 18, precision="fp16")) == [pk.Schedule(9, 0, 0, 0, 1)]
    # accumulator slots around the default (which targets about 512 row-pass workgroups up to 2^17 points:
    # 64 slots of 8 tiles at 2^12, capped at 64)
    small = {c.rowpass_slots for c in pk.schedule_candidates(pk.Instance(fft_len=1 << 12))
             if c.log2_n1 == 6 and c.single_pass == 2}
    assert small == {32, 64}
    # short transforms also list the single pass, with slots around 512 / n_pairs
    single = {c for c in pk.schedule_candidates(pk.Instance(fft_len=1 << 12)) if c.single_pass == 1}
    assert single == {pk.Schedule(6, 0, 0, 0, G, 1) for G in (64, 128, 256, 512)}  # default 2^20 / 2^12 = 256
    assert not any(c.single_pass == 1 for c in pk.schedule_candidates(pk.Instance(fft_len=1 << 13)))
    # tiny transform: only the split that keeps both passes >= 16 points
    assert {c.log2_n1 for c in pk.schedule_candidates(pk.Instance(fft_len=256))} == {4}


@pytest.mark.parametrize("sched", [pk.Schedule(3, 0, 0, 0), pk.Schedule(9, 4, 0, 0), pk.Schedule(9, 0, 2, 0),
                                   pk.Schedule(13, 0, 0, 0), pk.Schedule(9, 0, 0, 9), pk.Schedule(9, 0, 0, 0, 3),
                                   pk.Schedule(9, 0, 0, 0, 128)])
def test_scheduled_plan_rejects_unbuilt_schedules(sched):
    arr = (pk._Instance * 1)(pk.Instance(fft_len=1 << 18, bits=8).to_c())
    sarr = (pk._Schedule * 1)(sched.to_c())
    h = C.c_void_p()
    n = C.c_size_t()
    st = pk.lib().ps_plan_scheduled(arr, sarr, 1, C.byref(h), C.byref(n))
    assert pk.STATUS[st] == "PS_ERR_UNSUPPORTED", pk.lib().ps_last_error()
    assert not h.value


@pytest.mark.parametrize("hop", [0, 1024, 512, 256, 128])
def test_plan_accepts_hops_and_keeps_room_for_the_waiting_samples(hop):
    st0, h0, n0 = _plan()
    st, h, n = _plan(hop=hop)
    assert st0 == 0 and st == 0, pk.lib().ps_last_error()
    extra = 0 if hop in (0, 1024) else 2 * (1024 - hop) * 2 * 2 // 8  # two halves of N - hop two-bit samples, 2 streams
    assert n - n0 >= extra
    sb = C.c_size_t()
    assert pk.lib().ps_state_bytes(h, 0, C.byref(sb)) == 0
    sb0 = C.c_size_t()
    assert pk.lib().ps_state_bytes(h0, 0, C.byref(sb0)) == 0
    assert sb.value - sb0.value == extra // 2
    pk.lib().ps_destroy(h)
    pk.lib().ps_destroy(h0)


@pytest.mark.parametrize("window", ["hamming", "blackman"])
def test_plan_accepts_apodisation_windows(window):
    st, h, n = _plan(window=window)
    assert st == 0, pk.lib().ps_last_error()
    pk.lib().ps_destroy(h)
    st, h, n = _plan(window=window, fft_len=1 << 16, precision="fp16", accum="kahan32")
    assert st == 0, pk.lib().ps_last_error()
    pk.lib().ps_destroy(h)


def test_post_reduction_argument_errors():
    """Validation happens before any launch (dummy device addresses are never touched)."""
    L = pk.lib()
    p = C.c_void_p(1 << 20)
    assert pk.STATUS[L.ps_channel_average(p, 4, 1000, 3, None, p, None, None)] == "PS_ERR_SIZE"
    assert pk.STATUS[L.ps_channel_average(None, 4, 1024, 4, None, p, None, None)] == "PS_ERR_ARG"
    assert pk.STATUS[L.ps_channel_average(p, 70000, 1024, 4, None, p, None, None)] == "PS_ERR_ARG"
    assert L.ps_channel_average(p, 0, 1024, 4, None, p, None, None) == 0  # nothing to do
    n = C.c_size_t()
    assert L.ps_bandpass_work_bytes(131072, 128, 0.06, C.byref(n)) == 0
    n_int = -(-(131072 - 2 * 7864) // 128)
    assert n.value >= (n_int * 14 + (n_int + 3)) * 8
    assert pk.STATUS[L.ps_bandpass_work_bytes(131072, 16, 0.0, C.byref(n))] == "PS_ERR_UNSUPPORTED"
    assert pk.STATUS[L.ps_bandpass_work_bytes(500, 128, 0.06, C.byref(n))] == "PS_ERR_SIZE"  # 440 < 4 x 128
    assert pk.STATUS[L.ps_bandpass_work_bytes(131072, 2, 0.06, C.byref(n))] == "PS_ERR_ARG"
    assert pk.STATUS[L.ps_bandpass_work_bytes(131072, 128, 0.5, C.byref(n))] == "PS_ERR_ARG"
    assert pk.STATUS[L.ps_bandpass_fit(p, 131072, 128, 0.06, p, 16, p, None)] == "PS_ERR_WORKSPACE"

    assert pk.STATUS[L.ps_band_stats(p, 1, 0, p, None)] == "PS_ERR_ARG"
    lags = (C.c_int32 * 2)(1, 0)
    assert pk.STATUS[L.ps_allan(p, 100, 1, 1, 100, lags, 2, 1.0, 0, p, 1 << 20, p, None)] == "PS_ERR_ARG"
    assert pk.STATUS[L.ps_allan(p, 100, 1, 1, 100, lags, 0, 1.0, 0, p, 1 << 20, p, None)] == "PS_ERR_ARG"
    lags = (C.c_int32 * 1)(1)
    assert pk.STATUS[L.ps_allan(p, 100, 1, 1, 100, lags, 1, 0.0, 0, p, 1 << 20, p, None)] == "PS_ERR_ARG"
    nb = C.c_size_t()
    assert L.ps_allan_work_bytes(131072, 1, 30, 131072, 8, C.byref(nb)) == 0 and nb.value == 30 * 32 * 9 * 2 * 8
    assert L.ps_allan_work_bytes(1800, 4096, 4096, 1, 8, C.byref(nb)) == 0 and nb.value == 0  # side by side
    assert pk.STATUS[L.ps_allan(p, 131072, 1, 30, 131072, lags, 1, 1.0, 0, p, 16, p, None)] == "PS_ERR_WORKSPACE"


@pytest.mark.parametrize("n,sched,ok", [
    (1 << 12, pk.Schedule(0, 0, 0, 0, 0, 1), True),
    (1 << 12, pk.Schedule(0, 0, 0, 0, 4096, 1), True),
    (1 << 12, pk.Schedule(0, 0, 0, 0, 8192, 1), True),
    (1 << 12, pk.Schedule(0, 0, 0, 0, 16384, 1), False),
    (1 << 12, pk.Schedule(0, 16, 0, 0, 0, 1), False),    # the single pass has no column tiles
    (1 << 12, pk.Schedule(0, 16, 0, 0, 0, 0), False),    # default for 2^12 is the single pass
    (1 << 12, pk.Schedule(0, 16, 0, 0, 0, 2), True),
    (1 << 13, pk.Schedule(0, 0, 0, 0, 0, 1), False),     # above 2^12
    (1 << 12, pk.Schedule(0, 0, 0, 0, 0, 3), False),
])
def test_single_pass_schedules(n, sched, ok):
    arr = (pk._Instance * 1)(pk.Instance(fft_len=n, bits=8).to_c())
    sarr = (pk._Schedule * 1)(sched.to_c())
    h = C.c_void_p()
    nb = C.c_size_t()
    st = pk.lib().ps_plan_scheduled(arr, sarr, 1, C.byref(h), C.byref(nb))
    assert (st == 0) == ok, pk.lib().ps_last_error()
    if h.value:
        pk.lib().ps_destroy(h)


def test_learnable_window_needs_short_passes():
    """The adjoint's passes are built up to 512 points: a learnable-window instance may not take a split with
    a longer pass (2^18 as 1024 x 256 or 256 x 1024 is rejected, 512 x 512 accepted)."""
    inst = pk.Instance(fft_len=1 << 18, bits=8, window="taps", n_taps=64)
    for sched, ok in ((pk.Schedule(9), True), (pk.Schedule(10), False), (pk.Schedule(8), False)):
        arr = (pk._Instance * 1)(inst.to_c())
        sarr = (pk._Schedule * 1)(sched.to_c())
        h = C.c_void_p()
        n = C.c_size_t()
        st = pk.lib().ps_plan_scheduled(arr, sarr, 1, C.byref(h), C.byref(n))
        assert (st == 0) == ok, (sched, pk.lib().ps_last_error())
        if h.value:
            pk.lib().ps_destroy(h)


def test_instances_share_one_inter_pass_buffer():
    """The inter-pass buffer is one region for the whole plan: the largest instance's chunk, and at least the
    128 MiB of a grouped sub-batch when the plan has several instances (host-side sizing, no GPU)."""
    paper = pk.Instance(fft_len=1 << 18, bits=8)
    one = pk.plan_workspace_bytes([paper])
    t18 = 128 * (1 << 18) * 8  # default chunk of 2^25 points (128 frames of 2^18), one pair: 256 MiB
    assert one >= t18
    many = pk.plan_workspace_bytes([paper] * 64)
    per_inst = one - t18  # everything an instance owns besides the shared buffer (tables, accumulators, ...)
    assert many < t18 + 64 * (per_inst + (1 << 20))  # one buffer, not 64 (which would be > 8 GiB)
    mixed = pk.plan_workspace_bytes([paper, pk.Instance(fft_len=1 << 20, bits=2), pk.Instance(fft_len=1 << 12)])
    t20 = 64 * (1 << 20) * 8  # 512 MiB: the largest chunk sets the buffer
    assert t20 <= mixed < t20 + 3 * (per_inst + (64 << 20))
