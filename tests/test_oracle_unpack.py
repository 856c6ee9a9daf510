"""Oracle pins for the unpack step (data translation of 2/4/8-bit codes, Sec. 2 / Fig. 2 caption)."""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "unpack_cases.txt")


def _golden_cases():
    cases = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split(":")
            parts = lhs.split()
            bits, S = int(parts[0]), int(parts[1])
            raw = bytes.fromhex("".join(parts[2:]))
            levels = [float(v) for v in rhs.split()]
            cases.append((bits, S, np.frombuffer(raw, dtype=np.uint8), levels))
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: f"b{c[0]}s{c[1]}-{c[2].tobytes().hex()}")
def test_hand_decoded_cases(case):
    bits, S, packed, levels = case
    n_items = len(levels)
    T = n_items // S
    out = oracle.unpack(packed, bits, S, T)       # [S][T]
    got = out.T.reshape(-1)                        # time-major
    assert got.tolist() == levels


# per-code levels written out by hand (odd levels, offset binary)
LEVELS2 = [-3.0, -1.0, 1.0, 3.0]
LEVELS4 = [-15.0, -13.0, -11.0, -9.0, -7.0, -5.0, -3.0, -1.0, 1.0, 3.0, 5.0, 7.0, 9.0, 11.0, 13.0, 15.0]


@pytest.mark.parametrize("bits,table", [(2, LEVELS2), (4, LEVELS4)])
@pytest.mark.parametrize("S", [2, 4])
def test_every_byte_value_roundtrips_through_the_packer(bits, table, S):
    """Every byte value: codes packed by the sampler emulator decode to the hand-listed levels."""
    per = 8 // bits
    n_bytes = 256
    codes = np.zeros(n_bytes * per, dtype=np.uint8)
    for v in range(256):
        for i in range(per):
            codes[v * per + i] = (v >> (i * bits)) & ((1 << bits) - 1)
    codes = codes.reshape(-1, S)
    packed = synth.pack_codes(codes, bits)
    assert packed.tolist() == list(range(256))
    out = oracle.unpack(packed, bits, S, codes.shape[0])
    expect = np.array([[table[c] for c in row] for row in codes], dtype=np.float64)
    assert np.array_equal(out.T, expect)


def test_int8_every_value():
    codes = np.arange(256, dtype=np.uint8).reshape(-1, 2)
    out = oracle.unpack(synth.pack_codes(codes, 8), 8, 2, codes.shape[0])
    expect = np.arange(256, dtype=np.int64)
    expect = np.where(expect >= 128, expect - 256, expect).reshape(-1, 2).astype(np.float64)
    assert np.array_equal(out.T, expect)


@pytest.mark.parametrize("bits", [2, 4, 8])
def test_level_order_follows_the_analog_value(bits):
    """The decoded level is a non-decreasing function of the sampled voltage and has its sign."""
    x = np.linspace(-5, 5, 4000)
    xs = x * (16.0 if bits == 8 else 1.0)
    codes = synth.quantize(np.stack([xs, -xs], axis=1), bits)
    lv = oracle.unpack(synth.pack_codes(codes, bits), bits, 2, x.size)
    assert np.all(np.diff(lv[0]) >= 0) and np.all(np.diff(lv[1]) <= 0)
    nz = np.abs(xs) > (0.5 if bits == 8 else 1e-9)
    assert np.all(np.sign(lv[0][nz]) == np.sign(xs[nz]))


def test_float32_format_is_exact():
    rng = np.random.default_rng(5)
    v = rng.standard_normal((100, 2)).astype(np.float32)
    out = oracle.unpack(synth.pack_codes(v, 32), 32, 2, 100)
    assert np.array_equal(out.T, v.astype(np.float64))
